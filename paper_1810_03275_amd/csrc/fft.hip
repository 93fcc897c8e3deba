// Fourier-domain preconditioner (thesis §4.3, §4.3.1, §4.4) on gfx950.
//
// x = base + F^{-1}(m * F(y)) for a real image y (n x n, n = 2^a 3^b, even)
// and a real multiplier m that is even in each frequency.  Three kernels:
//   row pass     : two real rows packed as one complex row, mixed-radix
//                  (4/2/3) Stockham FFT in LDS, split into the two half
//                  spectra, written column-major: spec[k1][j];
//   column pass  : per k1, FFT along j, multiply by m[k1][k2], inverse FFT;
//   inverse rows : rebuild the two Hermitian spectra as one complex row,
//                  inverse FFT, real/imaginary parts are the two output rows.
// Twiddles exp(-2 pi i m/n) are precomputed in FP64 and stored as FP32.
#include <cmath>

#include "common.hpp"

namespace ctpd {

__device__ inline float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// One radix-R Stockham pass over `nrows` rows of length L (row stride L):
// reads a, writes b.  Ns is the length of the sub-transforms already done.
template <int R, bool INV>
__device__ inline void fft_pass(const float2 *a, float2 *b, int nrows, int L, int Ns,
                                const float2 *__restrict__ tw) {
  const int nbf = L / R;
  const int step = L / (Ns * R);
  const float sgn = INV ? 1.f : -1.f;  // forward kernel exp(-i ...)
  // exact small-integer quotients via a float reciprocal (operands < 2^13)
  const float inv_nbf = 1.0f / (float)nbf, inv_ns = 1.0f / (float)Ns;
  for (int t = threadIdx.x; t < nrows * nbf; t += blockDim.x) {
    const int row = (int)(((float)t + 0.5f) * inv_nbf);
    const int jj = t - row * nbf;
    const float2 *in = a + row * L;
    float2 *out = b + row * L;
    const int jq = (int)(((float)jj + 0.5f) * inv_ns);  // jj / Ns
    const int k = jj - jq * Ns;
    float2 v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = in[jj + r * nbf];
#pragma unroll
    for (int r = 1; r < R; ++r) {
      float2 w = tw[k * r * step];
      if (INV) w.y = -w.y;
      v[r] = cmul(v[r], w);
    }
    if (R == 2) {
      const float2 x0 = v[0], x1 = v[1];
      v[0] = make_float2(x0.x + x1.x, x0.y + x1.y);
      v[1] = make_float2(x0.x - x1.x, x0.y - x1.y);
    } else if (R == 4) {
      const float2 x0 = v[0], x1 = v[1], x2 = v[2 % R], x3 = v[3 % R];
      const float2 s02 = make_float2(x0.x + x2.x, x0.y + x2.y);
      const float2 d02 = make_float2(x0.x - x2.x, x0.y - x2.y);
      const float2 s13 = make_float2(x1.x + x3.x, x1.y + x3.y);
      const float2 d13 = make_float2(x1.x - x3.x, x1.y - x3.y);
      const float2 rd = make_float2(-sgn * d13.y, sgn * d13.x);  // (sgn i) d13
      v[0] = make_float2(s02.x + s13.x, s02.y + s13.y);
      v[1] = make_float2(d02.x + rd.x, d02.y + rd.y);
      v[2 % R] = make_float2(s02.x - s13.x, s02.y - s13.y);
      v[3 % R] = make_float2(d02.x - rd.x, d02.y - rd.y);
    } else {  // R == 3
      const float2 x0 = v[0], x1 = v[1], x2 = v[2 % R];
      const float h = 0.86602540378443864676f;  // sqrt(3)/2
      const float2 s = make_float2(x1.x + x2.x, x1.y + x2.y);
      const float2 d = make_float2(x1.x - x2.x, x1.y - x2.y);
      const float2 m = make_float2(x0.x - 0.5f * s.x, x0.y - 0.5f * s.y);
      const float2 rd = make_float2(-sgn * h * d.y, sgn * h * d.x);  // (sgn i sqrt(3)/2) d
      v[0] = make_float2(x0.x + s.x, x0.y + s.y);
      v[1] = make_float2(m.x + rd.x, m.y + rd.y);
      v[2 % R] = make_float2(m.x - rd.x, m.y - rd.y);
    }
    const int base = jq * Ns * R + k;
#pragma unroll
    for (int r = 0; r < R; ++r) out[base + r * Ns] = v[r];
  }
}

// Stockham FFT of `nrows` rows of length L held in LDS buffer a (row stride
// L); b is the ping-pong buffer.  Returns the buffer holding the result.
// INV selects the inverse (conjugate) transform, unnormalized.
template <bool INV>
__device__ float2 *fft_rows(float2 *a, float2 *b, int nrows, const FftPlan &pl,
                            const float2 *__restrict__ tw) {
  const int L = pl.L;
  int Ns = 1;
  for (int ps = 0; ps < pl.npass; ++ps) {
    const int R = pl.radix[ps];
    if (R == 4)
      fft_pass<4, INV>(a, b, nrows, L, Ns, tw);
    else if (R == 2)
      fft_pass<2, INV>(a, b, nrows, L, Ns, tw);
    else
      fft_pass<3, INV>(a, b, nrows, L, Ns, tw);
    __syncthreads();
    float2 *tmp = a;
    a = b;
    b = tmp;
    Ns *= R;
  }
  return a;
}

// Row pass: rows [2 rp0, 2 rp0 + 2 RP) of y -> spec[k1][j], k1 in [0, n/2].
__global__ __launch_bounds__(256) void k_fft_rows_fwd(const float *__restrict__ y, int n,
                                                      int RP, FftPlan pl,
                                                      const float2 *__restrict__ tw,
                                                      float2 *__restrict__ spec) {
  extern __shared__ float2 sm[];
  float2 *a = sm;
  float2 *b = sm + RP * n;
  const int pair0 = blockIdx.x * RP;
  const int npair = min(RP, n / 2 - pair0);
  y += (size_t)blockIdx.y * n * n;  // problem blockIdx.y of a batch
  spec += (size_t)blockIdx.y * (n / 2 + 1) * n;
  for (int t = threadIdx.x; t < npair * n; t += blockDim.x) {
    const int pr = (int)(((float)t + 0.5f) / (float)n), i = t - pr * n;
    const int j = 2 * (pair0 + pr);
    a[t] = make_float2(y[(size_t)j * n + i], y[(size_t)(j + 1) * n + i]);
  }
  __syncthreads();
  float2 *z = fft_rows<false>(a, b, npair, pl, tw);
  const int half = n / 2 + 1;
  const int w = 2 * npair;
  for (int t = threadIdx.x; t < half * w; t += blockDim.x) {
    const int k = t / w, c = t - k * w;
    const int pr = c >> 1;
    const float2 Zk = z[pr * n + k];
    const float2 Zm = z[pr * n + ((n - k) % n)];
    float2 out;
    if ((c & 1) == 0) {  // X = (Z[k] + conj(Z[-k]))/2
      out = make_float2(0.5f * (Zk.x + Zm.x), 0.5f * (Zk.y - Zm.y));
    } else {             // Y = (Z[k] - conj(Z[-k]))/(2i)
      out = make_float2(0.5f * (Zk.y + Zm.y), -0.5f * (Zk.x - Zm.x));
    }
    spec[(size_t)k * n + 2 * pair0 + c] = out;
  }
}

// Column pass: per k1, spec[k1][:] <- IFFT( m[k1][:] * FFT(spec[k1][:]) ).
__global__ __launch_bounds__(256) void k_fft_cols(float2 *__restrict__ spec, int n, int CP,
                                                  FftPlan pl, const float2 *__restrict__ tw,
                                                  const float *__restrict__ mult) {
  extern __shared__ float2 sm[];
  float2 *a = sm;
  float2 *b = sm + CP * n;
  const int half = n / 2 + 1;
  const int k10 = blockIdx.x * CP;
  const int ncol = min(CP, half - k10);
  spec += (size_t)blockIdx.y * half * n;
  for (int t = threadIdx.x; t < ncol * n; t += blockDim.x) a[t] = spec[(size_t)k10 * n + t];
  __syncthreads();
  float2 *z = fft_rows<false>(a, b, ncol, pl, tw);
  float2 *other = (z == a) ? b : a;
  for (int t = threadIdx.x; t < ncol * n; t += blockDim.x) {
    const float m = mult[(size_t)k10 * n + t];
    z[t] = make_float2(m * z[t].x, m * z[t].y);
  }
  __syncthreads();
  z = fft_rows<true>(z, other, ncol, pl, tw);
  for (int t = threadIdx.x; t < ncol * n; t += blockDim.x) spec[(size_t)k10 * n + t] = z[t];
}

// Inverse row pass: out[j][i] = (base ? base[j][i] : 0) + x_j[i].
__global__ __launch_bounds__(256) void k_fft_rows_inv(const float2 *__restrict__ spec, int n,
                                                      int RP, FftPlan pl,
                                                      const float2 *__restrict__ tw,
                                                      const float *__restrict__ base,
                                                      float *__restrict__ out) {
  extern __shared__ float2 sm[];
  float2 *a = sm;
  float2 *b = sm + RP * n;
  const int pair0 = blockIdx.x * RP;
  const int npair = min(RP, n / 2 - pair0);
  const int half = n / 2 + 1;
  spec += (size_t)blockIdx.y * half * n;
  if (base != nullptr) base += (size_t)blockIdx.y * n * n;
  out += (size_t)blockIdx.y * n * n;
  for (int t = threadIdx.x; t < npair * n; t += blockDim.x) {
    const int pr = t / n, k = t - pr * n;
    const int j = 2 * (pair0 + pr);
    float2 X, Y;
    if (k < half) {
      X = spec[(size_t)k * n + j];
      Y = spec[(size_t)k * n + j + 1];
    } else {
      const int km = n - k;
      X = spec[(size_t)km * n + j];
      Y = spec[(size_t)km * n + j + 1];
      X.y = -X.y;
      Y.y = -Y.y;
    }
    a[t] = make_float2(X.x - Y.y, X.y + Y.x);  // X + i Y
  }
  __syncthreads();
  float2 *z = fft_rows<true>(a, b, npair, pl, tw);
  for (int t = threadIdx.x; t < npair * n; t += blockDim.x) {
    const int pr = t / n, i = t - pr * n;
    const int j = 2 * (pair0 + pr);
    const size_t o0 = (size_t)j * n + i, o1 = o0 + n;
    const float2 v = z[t];
    out[o0] = (base ? base[o0] : 0.f) + v.x;
    out[o1] = (base ? base[o1] : 0.f) + v.y;
  }
}

// Rows (pairs) per workgroup: at least ~256 workgroups, at most 64 KB of LDS.
static int rows_per_block(int n) {
  int rp = 4096 / n;  // keep 2 * RP * n * 8 bytes <= 64 KB
  if (rp < 1) rp = 1;
  if (rp > 4) rp = 4;
  while (rp > 1 && (n / 2) / rp < 256) rp /= 2;
  return rp;
}

int launch_apply_mult(const ct_precond *pc, const float *mult, const float *y,
                      const float *base, float *out, hipStream_t s, int nb, float2 *spec) {
  const int n = pc->n;
  int RP = rows_per_block(n);
  // a batch fills the chip with its problems: fewer, larger row blocks
  while (nb > 1 && RP < 4 && 2 * RP * n * 8 <= 65536 && (n / 2) / (2 * RP) * nb >= 512) RP *= 2;
  const int half = n / 2 + 1;
  if (nb < 1 || (nb > 1 && spec == nullptr)) {
    set_error("preconditioner: batch needs its own spectrum buffer");
    return CT_E_INVALID;
  }
  if (spec == nullptr) spec = pc->d_spec;
  const size_t lds = 2 * sizeof(float2) * (size_t)RP * n;
  hipLaunchKernelGGL(k_fft_rows_fwd, dim3((n / 2 + RP - 1) / RP, nb), dim3(256), lds, s, y, n,
                     RP, pc->fp, pc->d_tw, spec);
  CT_TRY_HIP(hipGetLastError());
  const int CP = RP;
  hipLaunchKernelGGL(k_fft_cols, dim3((half + CP - 1) / CP, nb), dim3(256), lds, s, spec, n, CP,
                     pc->fp, pc->d_tw, mult);
  CT_TRY_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_fft_rows_inv, dim3((n / 2 + RP - 1) / RP, nb), dim3(256), lds, s, spec,
                     n, RP, pc->fp, pc->d_tw, base, out);
  CT_TRY_HIP(hipGetLastError());
  return CT_OK;
}

bool fft_factor(int L, FftPlan *fp) {
  fp->L = L;
  fp->npass = 0;
  int m = L;
  while (m % 4 == 0) { fp->radix[fp->npass++] = 4; m /= 4; }
  while (m % 2 == 0) { fp->radix[fp->npass++] = 2; m /= 2; }
  while (m % 3 == 0) { fp->radix[fp->npass++] = 3; m /= 3; }
  return m == 1 && fp->npass <= 24;
}

}  // namespace ctpd
