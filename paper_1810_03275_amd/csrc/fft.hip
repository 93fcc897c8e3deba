// Fourier-domain preconditioner (thesis §4.3, §4.3.1, §4.4) on gfx950.
//
// x = base + F^{-1}(m * F(y)) for a real image y (n x n, n = 2^a 3^b, even)
// and a real multiplier m that is even in each frequency.  Three kernels:
//   row pass     : two real rows packed as one complex row, mixed-radix
//                  (8/4/3/2) Stockham FFT in LDS, split into the two half
//                  spectra, written column-major: spec[k1][j];
//   column pass  : per k1, FFT along j, multiply by m[k1][k2], inverse FFT;
//   inverse rows : rebuild the two Hermitian spectra as one complex row,
//                  inverse FFT, real/imaginary parts are the two output rows.
// Twiddles exp(-2 pi i m/n) are precomputed in FP64 and stored as FP32.
#include <algorithm>
#include <cmath>
#include <type_traits>

#include "common.hpp"

namespace ctpd {

// Threads per workgroup of every FFT kernel (a compile-time constant: the
// strided loops use it instead of reading the dispatch's workgroup size).
constexpr int kFftThreads = 256;

__device__ inline float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// Radix-4 DFT in place, kernel exp(sgn 2 pi i jk / 4).
__device__ inline void dft4(float2 &v0, float2 &v1, float2 &v2, float2 &v3, float sgn) {
  const float2 s02 = make_float2(v0.x + v2.x, v0.y + v2.y);
  const float2 d02 = make_float2(v0.x - v2.x, v0.y - v2.y);
  const float2 s13 = make_float2(v1.x + v3.x, v1.y + v3.y);
  const float2 d13 = make_float2(v1.x - v3.x, v1.y - v3.y);
  const float2 rd = make_float2(-sgn * d13.y, sgn * d13.x);  // (sgn i) d13
  v0 = make_float2(s02.x + s13.x, s02.y + s13.y);
  v1 = make_float2(d02.x + rd.x, d02.y + rd.y);
  v2 = make_float2(s02.x - s13.x, s02.y - s13.y);
  v3 = make_float2(d02.x - rd.x, d02.y - rd.y);
}

// One radix-R Stockham pass over `nrows` rows of length L (row stride L):
// reads a, writes b.  Ns is the length of the sub-transforms already done.
// tw holds exp(-2 pi i m / L), m < L (in LDS or global memory).
template <int R, bool INV>
__device__ inline void fft_pass(const float2 *a, float2 *b, int nrows, int L, int Ns,
                                const float2 *tw) {
  const int nbf = L / R;
  const int step = L / (Ns * R);
  const float sgn = INV ? 1.f : -1.f;  // forward kernel exp(-i ...)
  // exact small-integer quotients via a float reciprocal (operands < 2^13)
  const float inv_nbf = 1.0f / (float)nbf, inv_ns = 1.0f / (float)Ns;
  for (int t = threadIdx.x; t < nrows * nbf; t += kFftThreads) {
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
    if constexpr (R == 2) {
      const float2 x0 = v[0], x1 = v[1];
      v[0] = make_float2(x0.x + x1.x, x0.y + x1.y);
      v[1] = make_float2(x0.x - x1.x, x0.y - x1.y);
    } else if constexpr (R == 4) {
      dft4(v[0], v[1], v[2], v[3], sgn);
    } else if constexpr (R == 8) {
      // a_j = x_j + x_{j+4} and b_j = (x_j - x_{j+4}) w8^j (w8 = exp(sgn i pi / 4));
      // the even outputs are the DFT-4 of a, the odd outputs that of b
      const float c = 0.70710678118654752440f;  // sqrt(2)/2
      float2 a4[4], b4[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        a4[j] = make_float2(v[j].x + v[j + 4].x, v[j].y + v[j + 4].y);
        b4[j] = make_float2(v[j].x - v[j + 4].x, v[j].y - v[j + 4].y);
      }
      b4[1] = make_float2(c * (b4[1].x - sgn * b4[1].y), c * (b4[1].y + sgn * b4[1].x));
      b4[2] = make_float2(-sgn * b4[2].y, sgn * b4[2].x);
      b4[3] = make_float2(-c * (b4[3].x + sgn * b4[3].y), c * (sgn * b4[3].x - b4[3].y));
      dft4(a4[0], a4[1], a4[2], a4[3], sgn);
      dft4(b4[0], b4[1], b4[2], b4[3], sgn);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        v[2 * j] = a4[j];
        v[2 * j + 1] = b4[j];
      }
    } else {  // R == 3
      static_assert(R == 3, "radix 2, 3, 4 or 8");
      const float2 x0 = v[0], x1 = v[1], x2 = v[2];
      const float h = 0.86602540378443864676f;  // sqrt(3)/2
      const float2 s = make_float2(x1.x + x2.x, x1.y + x2.y);
      const float2 d = make_float2(x1.x - x2.x, x1.y - x2.y);
      const float2 m = make_float2(x0.x - 0.5f * s.x, x0.y - 0.5f * s.y);
      const float2 rd = make_float2(-sgn * h * d.y, sgn * h * d.x);  // (sgn i sqrt(3)/2) d
      v[0] = make_float2(x0.x + s.x, x0.y + s.y);
      v[1] = make_float2(m.x + rd.x, m.y + rd.y);
      v[2] = make_float2(m.x - rd.x, m.y - rd.y);
    }
    const int base = jq * Ns * R + k;
#pragma unroll
    for (int r = 0; r < R; ++r) out[base + r * Ns] = v[r];
  }
}

// Value of v in another lane of the same quad, chosen by the DPP quad
// permutation CTRL (0x4E reads lane ^ 2, 0xB1 lane ^ 1).  All four lanes of
// the quad must be active.
template <int CTRL>
__device__ inline float quad_perm(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, false));
}

// One radix-8 Stockham pass, the same transform as fft_pass<8>, with every
// butterfly spread over the four lanes of a quad, for power-of-two lengths
// L = 2^lgL (Ns = 2^lgNs).  Lane q takes inputs q and q + 4 and forms
// a_q = x_q + x_{q+4} and b_q = (x_q - x_{q+4}) w8^q; the two 4-point DFTs of
// a and b (the even and the odd outputs) then run across the quad as two
// radix-2 steps, with partners q ^ 2 and q ^ 1, each one FMA with a lane sign
// (+1 keeps the sum, -1 the difference).  A pass of L/8 butterflies keeps four
// times as many lanes busy, with no lane-dependent branches.
template <bool INV>
__device__ inline void fft_pass8_quad(const float2 *a, float2 *b, int nrows, int lgL, int lgNs,
                                      const float2 *tw) {
  const int lgnbf = lgL - 3;  // L/8 butterflies per row
  const int lgstep = lgL - lgNs - 3;  // twiddle stride L / (8 Ns)
  const float sgn = INV ? 1.f : -1.f;
  const float c = 0.70710678118654752440f;  // sqrt(2)/2
  // kFftThreads is a multiple of 4, so a quad's lanes share t >> 2 in every
  // iteration and leave the loop together
  const int q = threadIdx.x & 3;
  const float2 w8 = q == 0   ? make_float2(1.f, 0.f)
                    : q == 1 ? make_float2(c, sgn * c)
                    : q == 2 ? make_float2(0.f, sgn)
                             : make_float2(-c, sgn * c);  // exp(sgn i pi q / 4)
  const float s1 = q < 2 ? 1.f : -1.f, s2 = (q & 1) ? -1.f : 1.f;
  const bool rot = q == 3;  // the odd difference of the first step times (sgn i)
  const int p = ((q & 1) << 1) | (q >> 1);  // the 4-point output lane q ends with
  const int mj = (1 << lgnbf) - 1, mk = (1 << lgNs) - 1;
  for (int t = threadIdx.x; t < (nrows << (lgnbf + 2)); t += kFftThreads) {
    const int bf = t >> 2;
    const int row = bf >> lgnbf, jj = bf & mj;
    const int jq = jj >> lgNs, k = jj & mk;
    const float2 *in = a + (row << lgL) + jj;
    float2 x0 = in[q << lgnbf], x1 = in[(q + 4) << lgnbf];
    float2 w0 = tw[(k * q) << lgstep], w1 = tw[(k * (q + 4)) << lgstep];  // tw[0] = 1
    if (INV) {
      w0.y = -w0.y;
      w1.y = -w1.y;
    }
    x0 = cmul(x0, w0);
    x1 = cmul(x1, w1);
    float2 av = make_float2(x0.x + x1.x, x0.y + x1.y);
    float2 bv = cmul(make_float2(x0.x - x1.x, x0.y - x1.y), w8);
    {  // partner q ^ 2
      const float2 ap = make_float2(quad_perm<0x4E>(av.x), quad_perm<0x4E>(av.y));
      const float2 bp = make_float2(quad_perm<0x4E>(bv.x), quad_perm<0x4E>(bv.y));
      av = make_float2(fmaf(s1, av.x, ap.x), fmaf(s1, av.y, ap.y));
      bv = make_float2(fmaf(s1, bv.x, bp.x), fmaf(s1, bv.y, bp.y));
    }
    if (rot) {
      av = make_float2(-sgn * av.y, sgn * av.x);
      bv = make_float2(-sgn * bv.y, sgn * bv.x);
    }
    {  // partner q ^ 1
      const float2 ap = make_float2(quad_perm<0xB1>(av.x), quad_perm<0xB1>(av.y));
      const float2 bp = make_float2(quad_perm<0xB1>(bv.x), quad_perm<0xB1>(bv.y));
      av = make_float2(fmaf(s2, av.x, ap.x), fmaf(s2, av.y, ap.y));
      bv = make_float2(fmaf(s2, bv.x, bp.x), fmaf(s2, bv.y, bp.y));
    }
    // output 2p of the 8-point DFT is the a-DFT's p, output 2p + 1 the b-DFT's
    float2 *out = b + (row << lgL) + (jq << (lgNs + 3)) + k;
    out[(2 * p) << lgNs] = av;
    out[(2 * p + 1) << lgNs] = bv;
  }
}

// Stockham FFT of `nrows` rows of length L held in LDS buffer a (row stride
// L); b is the ping-pong buffer.  Returns the buffer holding the result.
// INV selects the inverse (conjugate) transform, unnormalized.
template <bool INV>
__device__ float2 *fft_rows(float2 *a, float2 *b, int nrows, const FftPlan &pl,
                            const float2 *tw) {
  const int L = pl.L;
  int Ns = 1;
  for (int ps = 0; ps < pl.npass; ++ps) {
    const int R = (int)((pl.code >> (4 * ps)) & 15u);
    if (R == 8 && pl.quad8)
      fft_pass8_quad<INV>(a, b, nrows, __builtin_ctz(L), __builtin_ctz(Ns), tw);
    else if (R == 8)
      fft_pass<8, INV>(a, b, nrows, L, Ns, tw);
    else if (R == 4)
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

// Row-pair index of workgroup b of G: workgroups are dealt to the 8 XCDs in
// turn, so consecutive row pairs -- which share the cache lines of the
// spectrum's columns -- are given to workgroups on one XCD (one L2).
__device__ inline int xcd_pair(int b, int G) {
  const int full = G & ~7;
  if (b >= full) return b;
  return (b & 7) * (full >> 3) + (b >> 3);
}

// A workgroup-strided loop over [0, total) whose loads are issued kIoBatch
// at a time (all before the first use), so that their latencies overlap.
constexpr int kIoBatch = 4;
template <typename Load, typename Use>
__device__ inline void batched(int total, Load load, Use use) {
  for (int t0 = threadIdx.x; t0 < total; t0 += kIoBatch * kFftThreads) {
    decltype(load(0)) r[kIoBatch];
#pragma unroll
    for (int u = 0; u < kIoBatch; ++u) {
      const int t = t0 + u * kFftThreads;
      if (t < total) r[u] = load(t);
    }
#pragma unroll
    for (int u = 0; u < kIoBatch; ++u) {
      const int t = t0 + u * kFftThreads;
      if (t < total) use(t, r[u]);
    }
  }
}

// Two neighbouring pixels (i0, i0 + 1; i0 even) of rows j and j + 1 of the
// deferred backprojection from DS = d.S partial images, with 8-byte loads:
// per pixel the slices' sum in slice order and the epilogue, the same
// operations in the same order as the stand-alone combine pass.  DS is a
// compile-time count so that all loads are in flight at once; row j + 1's
// lower neighbour in the field's second component is row j's own value.
template <int DS>
__device__ inline void deferred_two(const BpDeferred &d, int n, int i0, int j, float2 &r0,
                                    float2 &r1) {
  const size_t nn = (size_t)n * n, o0 = (size_t)j * n + i0, o1 = o0 + n;
  float2 a[DS], b[DS];
#pragma unroll
  for (int s = 0; s < DS; ++s) {
    a[s] = *reinterpret_cast<const float2 *>(d.part + s * nn + o0);
    b[s] = *reinterpret_cast<const float2 *>(d.part + s * nn + o1);
  }
  float2 u0 = a[0], u1 = b[0];
#pragma unroll
  for (int s = 1; s < DS; ++s) {
    u0.x += a[s].x;
    u0.y += a[s].y;
    u1.x += b[s].x;
    u1.y += b[s].y;
  }
  r0 = make_float2(d.c1 * u0.x, d.c1 * u0.y);
  r1 = make_float2(d.c1 * u1.x, d.c1 * u1.y);
  if (d.pfield != nullptr) {
    const float *p1 = d.pfield, *p2 = d.pfield + nn;
    const float2 q0 = *reinterpret_cast<const float2 *>(p1 + o0);
    const float2 q1 = *reinterpret_cast<const float2 *>(p1 + o1);
    const float l0 = i0 > 0 ? p1[o0 - 1] : 0.f, l1 = i0 > 0 ? p1[o1 - 1] : 0.f;
    const bool last = i0 + 1 >= n - 1;  // the second pixel is the row's last
    // d1 = (i < n - 1 ? p1[o] : 0) - (i > 0 ? p1[o - 1] : 0)
    const float d1a = q0.x - l0, d1b = (last ? 0.f : q0.y) - q0.x;
    const float e1a = q1.x - l1, e1b = (last ? 0.f : q1.y) - q1.x;
    // d2 = (j < n - 1 ? p2[o] : 0) - (j > 0 ? p2[o - n] : 0), rows j and j + 1
    const float2 w0 = *reinterpret_cast<const float2 *>(p2 + o0);
    const float2 w1 = *reinterpret_cast<const float2 *>(p2 + o1);
    const float2 wm = j > 0 ? *reinterpret_cast<const float2 *>(p2 + o0 - n) : make_float2(0.f, 0.f);
    const bool lastrow = j + 1 >= n - 1;
    const float d2a = w0.x - wm.x, d2b = w0.y - wm.y;
    const float e2a = (lastrow ? 0.f : w1.x) - w0.x, e2b = (lastrow ? 0.f : w1.y) - w0.y;
    const float k = d.c2 * d.inv_h;
    r0 = make_float2(fmaf(k, d1a + d2a, r0.x), fmaf(k, d1b + d2b, r0.y));
    r1 = make_float2(fmaf(k, e1a + e2a, r1.x), fmaf(k, e1b + e2b, r1.y));
  }
  if (d.base != nullptr) {
    const float2 g0 = *reinterpret_cast<const float2 *>(d.base + o0);
    const float2 g1 = *reinterpret_cast<const float2 *>(d.base + o1);
    r0 = make_float2(r0.x + g0.x, r0.y + g0.y);
    r1 = make_float2(r1.x + g1.x, r1.y + g1.y);
  }
  if (d.base2 != nullptr) {
    const float2 g0 = *reinterpret_cast<const float2 *>(d.base2 + o0);
    const float2 g1 = *reinterpret_cast<const float2 *>(d.base2 + o1);
    r0 = make_float2(r0.x - g0.x, r0.y - g0.y);
    r1 = make_float2(r1.x - g1.x, r1.y - g1.y);
  }
}

// Row pass: rows [2 rp0, 2 rp0 + 2 RP) of y -> spec[k1][j], k1 in [0, n/2].
// With DS > 0, y is the deferred backprojection yd of DS partial images
// (and epilogue), formed here as the rows are loaded.
template <bool TWL, int DS>
__global__ __launch_bounds__(kFftThreads) void k_fft_rows_fwd(const float *__restrict__ y, int n,
                                                      int RP, FftPlan pl,
                                                      const float2 *__restrict__ tw,
                                                      float2 *__restrict__ spec,
                                                      BpDeferred yd) {
  extern __shared__ float2 sm[];
  float2 *a = sm;
  float2 *b = sm + RP * n;
  // the twiddle table is copied into LDS by the same loops that load the
  // rows (its loads in flight with theirs: one memory round trip)
  float2 *twl = sm + 2 * RP * n;
  const float2 *twp = TWL ? twl : tw;
  const int pair0 = xcd_pair(blockIdx.x, gridDim.x) * RP;
  const int npair = min(RP, n / 2 - pair0);
  const size_t nn = (size_t)n * n;
  if (DS == 0) {
    y += blockIdx.y * nn;  // problem blockIdx.y of a batch
  } else {
    yd.part += blockIdx.y * yd.S * nn;
    if (yd.pfield != nullptr) yd.pfield += blockIdx.y * 2 * nn;
    if (yd.base != nullptr) yd.base += blockIdx.y * nn;
    if (yd.base2 != nullptr) yd.base2 += blockIdx.y * nn;
  }
  spec += (size_t)blockIdx.y * (n / 2 + 1) * n;
  if constexpr (DS > 0) {
    // two pixels of both rows per thread and step (n is even)
    const int hn = n / 2;
    const int tot = npair * hn;  // >= n / 2: twiddles t2 and t2 + tot cover [0, n)
    for (int t2 = threadIdx.x; t2 < tot; t2 += kFftThreads) {
      const int pr = (int)(((float)t2 + 0.5f) / (float)hn), i0 = 2 * (t2 - pr * hn);
      float2 w0 = make_float2(0.f, 0.f), w1 = w0;
      if (TWL && t2 < n) w0 = tw[t2];
      if (TWL && t2 + tot < n) w1 = tw[t2 + tot];
      float2 r0, r1;
      deferred_two<DS>(yd, n, i0, 2 * (pair0 + pr), r0, r1);
      a[pr * n + i0] = make_float2(r0.x, r1.x);
      a[pr * n + i0 + 1] = make_float2(r0.y, r1.y);
      if (TWL && t2 < n) twl[t2] = w0;
      if (TWL && t2 + tot < n) twl[t2 + tot] = w1;
    }
  } else {
    struct Ld {
      float2 v, w;
    };
    batched(
        npair * n,
        [&](int t) {
          const int pr = (int)(((float)t + 0.5f) / (float)n), i = t - pr * n;
          const int j = 2 * (pair0 + pr);
          Ld r{make_float2(y[(size_t)j * n + i], y[(size_t)(j + 1) * n + i]),
               make_float2(0.f, 0.f)};
          if (TWL && t < n) r.w = tw[t];
          return r;
        },
        [&](int t, Ld r) {
          a[t] = r.v;
          if (TWL && t < n) twl[t] = r.w;
        });
  }
  __syncthreads();
  float2 *z = fft_rows<false>(a, b, npair, pl, twp);
  const int half = n / 2 + 1;
  const int w = 2 * npair;
  for (int t = threadIdx.x; t < half * w; t += kFftThreads) {
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
// exp(sgn 2 pi i (j k1 mod n^2) / n^2) in FP64, rounded to FP32: the twiddle
// between the two passes of the length-n^2 DFT of a column-major vector
// (index j + n i; the row pass has transformed along i into frequency k1)
__device__ inline float2 flat_twiddle(int j, int k1, int n, float sgn) {
  const long long L = (long long)n * n;
  const long long q = ((long long)j * k1) % L;
  double sn, cs;
  sincospi(2.0 * (double)q / (double)L, &sn, &cs);
  return make_float2((float)cs, sgn * (float)sn);
}

template <bool TWL>
__global__ __launch_bounds__(kFftThreads) void k_fft_cols(float2 *__restrict__ spec, int n, int CP,
                                                  FftPlan pl, const float2 *__restrict__ tw,
                                                  const float *__restrict__ mult, int twist,
                                                  int mpre) {
  extern __shared__ float2 sm[];
  float2 *a = sm;
  float2 *b = sm + CP * n;
  // twiddles (TWL) and, with mpre, the multipliers are copied into LDS by
  // the loop that loads the columns: one memory round trip for all three
  float2 *twl = sm + 2 * CP * n;
  float *mb = reinterpret_cast<float *>(twl + (TWL ? n : 0));
  const float2 *twp = TWL ? twl : tw;
  const int half = n / 2 + 1;
  const int k10 = blockIdx.x * CP;
  const int ncol = min(CP, half - k10);
  spec += (size_t)blockIdx.y * half * n;
  struct Ld {
    float2 v, w;
    float m;
  };
  batched(
      ncol * n,
      [&](int t) {
        Ld r{spec[(size_t)k10 * n + t], make_float2(0.f, 0.f), 0.f};
        if (TWL && t < n) r.w = tw[t];
        if (mpre) r.m = mult[(size_t)k10 * n + t];
        return r;
      },
      [&](int t, Ld r) {
        float2 v = r.v;
        if (twist) {
          const int c = t / n;
          v = cmul(v, flat_twiddle(t - c * n, k10 + c, n, -1.f));
        }
        a[t] = v;
        if (TWL && t < n) twl[t] = r.w;
        if (mpre) mb[t] = r.m;
      });
  __syncthreads();
  float2 *z = fft_rows<false>(a, b, ncol, pl, twp);
  float2 *other = (z == a) ? b : a;
  if (mpre) {
    for (int t = threadIdx.x; t < ncol * n; t += kFftThreads) {
      const float m = mb[t];
      z[t] = make_float2(m * z[t].x, m * z[t].y);
    }
  } else {
    batched(ncol * n, [&](int t) { return mult[(size_t)k10 * n + t]; },
            [&](int t, float m) { z[t] = make_float2(m * z[t].x, m * z[t].y); });
  }
  __syncthreads();
  z = fft_rows<true>(z, other, ncol, pl, twp);
  for (int t = threadIdx.x; t < ncol * n; t += kFftThreads) {
    float2 v = z[t];
    if (twist) {
      const int c = t / n;
      v = cmul(v, flat_twiddle(t - c * n, k10 + c, n, 1.f));
    }
    spec[(size_t)k10 * n + t] = v;
  }
}

// Inverse row pass: out[j][i] = (base ? base[j][i] : 0) + x_j[i].
template <bool TWL>
__global__ __launch_bounds__(kFftThreads) void k_fft_rows_inv(const float2 *__restrict__ spec, int n,
                                                      int RP, FftPlan pl,
                                                      const float2 *__restrict__ tw,
                                                      const float *__restrict__ base,
                                                      float *__restrict__ out, int bpre) {
  extern __shared__ float2 sm[];
  float2 *a = sm;
  float2 *b = sm + RP * n;
  // twiddles (TWL) and, with bpre, the base rows are copied into LDS by the
  // loop that loads the spectrum: one memory round trip for all three
  float2 *twl = sm + 2 * RP * n;
  float2 *gb = twl + (TWL ? n : 0);
  const float2 *twp = TWL ? twl : tw;
  const int pair0 = xcd_pair(blockIdx.x, gridDim.x) * RP;
  const int npair = min(RP, n / 2 - pair0);
  const int half = n / 2 + 1;
  spec += (size_t)blockIdx.y * half * n;
  if (base != nullptr) base += (size_t)blockIdx.y * n * n;
  out += (size_t)blockIdx.y * n * n;
  const bool pre = bpre && base != nullptr;
  struct Ld {
    float4 xy;
    float2 w, g;
  };
  batched(
      npair * n,
      [&](int t) {
        const int pr = t / n, k = t - pr * n;
        const int j = 2 * (pair0 + pr);
        const int kk = k < half ? k : n - k;
        // X and Y of row pair j at frequency kk (contiguous in spec)
        Ld r{*reinterpret_cast<const float4 *>(spec + (size_t)kk * n + j), make_float2(0.f, 0.f),
             make_float2(0.f, 0.f)};
        if (TWL && t < n) r.w = tw[t];
        if (pre) {
          const size_t o0 = (size_t)j * n + k;  // pixel k of rows j, j + 1
          r.g = make_float2(base[o0], base[o0 + n]);
        }
        return r;
      },
      [&](int t, Ld r) {
        const int k = t - (t / n) * n;
        float2 X = make_float2(r.xy.x, r.xy.y), Y = make_float2(r.xy.z, r.xy.w);
        if (k >= half) {  // Hermitian symmetry: conjugates of frequency n - k
          X.y = -X.y;
          Y.y = -Y.y;
        }
        a[t] = make_float2(X.x - Y.y, X.y + Y.x);  // X + i Y
        if (TWL && t < n) twl[t] = r.w;
        if (pre) gb[t] = r.g;
      });
  __syncthreads();
  float2 *z = fft_rows<true>(a, b, npair, pl, twp);
  if (pre) {
    for (int t = threadIdx.x; t < npair * n; t += kFftThreads) {
      const int pr = t / n, i = t - pr * n;
      const size_t o0 = (size_t)(2 * (pair0 + pr)) * n + i;
      const float2 v = z[t], g = gb[t];
      out[o0] = g.x + v.x;
      out[o0 + n] = g.y + v.y;
    }
    return;
  }
  batched(
      npair * n,
      [&](int t) {
        const int pr = t / n, i = t - pr * n;
        const size_t o0 = (size_t)(2 * (pair0 + pr)) * n + i;
        return base ? make_float2(base[o0], base[o0 + n]) : make_float2(0.f, 0.f);
      },
      [&](int t, float2 b0) {
        const int pr = t / n, i = t - pr * n;
        const size_t o0 = (size_t)(2 * (pair0 + pr)) * n + i;
        const float2 v = z[t];
        out[o0] = b0.x + v.x;
        out[o0 + n] = b0.y + v.y;
      });
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
                      const float *base, float *out, hipStream_t s, int nb, float2 *spec,
                      const BpDeferred *ydef) {
  const BpDeferred yd = ydef ? *ydef : BpDeferred{};
  const int DS = (ydef != nullptr && yd.part != nullptr) ? yd.S : 0;  // the deferred form wins
  if ((DS == 0 && y == nullptr) || (DS != 0 && !deferrable_slices(DS))) {
    set_error("preconditioner: no input image, or an unsupported slice count");
    return CT_E_INVALID;
  }
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
  const size_t rows_lds = 2 * sizeof(float2) * (size_t)RP * n;
  const bool twl = rows_lds + sizeof(float2) * n <= 65536;
  const size_t lds = rows_lds + (twl ? sizeof(float2) * n : 0);
  // the column pass's multipliers and the inverse pass's base rows go to LDS
  // with the loads they share a round trip with, where they fit
  const size_t lds_cols = lds + sizeof(float) * (size_t)RP * n;
  const size_t lds_inv = lds + sizeof(float2) * (size_t)RP * n;
  const int mpre = lds_cols <= 65536, bpre = lds_inv <= 65536;
  const dim3 block(kFftThreads);
  const int CP = RP;
  const dim3 grow((n / 2 + RP - 1) / RP, nb);
  auto rows_fwd = [&](auto twl_c) {
    constexpr bool T = decltype(twl_c)::value;
    switch (DS) {
#define CT_ROWS_FWD(K)                                                                     \
  case K:                                                                                  \
    hipLaunchKernelGGL((k_fft_rows_fwd<T, K>), grow, block, lds, s, y, n, RP, pc->fp,      \
                       pc->d_tw, spec, yd);                                                \
    break;
      CT_ROWS_FWD(0)
      CT_ROWS_FWD(2)
      CT_ROWS_FWD(3)
      CT_ROWS_FWD(4)
      CT_ROWS_FWD(5)
      CT_ROWS_FWD(6)
      CT_ROWS_FWD(7)
      CT_ROWS_FWD(8)
      CT_ROWS_FWD(16)
#undef CT_ROWS_FWD
    }
  };
  if (twl) {
    rows_fwd(std::true_type{});
    hipLaunchKernelGGL(k_fft_cols<true>, dim3((half + CP - 1) / CP, nb), block,
                       mpre ? lds_cols : lds, s, spec, n, CP, pc->fp, pc->d_tw, mult, pc->twist,
                       mpre);
    hipLaunchKernelGGL(k_fft_rows_inv<true>, dim3((n / 2 + RP - 1) / RP, nb), block,
                       bpre ? lds_inv : lds, s, spec, n, RP, pc->fp, pc->d_tw, base, out, bpre);
  } else {
    rows_fwd(std::false_type{});
    hipLaunchKernelGGL(k_fft_cols<false>, dim3((half + CP - 1) / CP, nb), block,
                       mpre ? lds_cols : lds, s, spec, n, CP, pc->fp, pc->d_tw, mult, pc->twist,
                       mpre);
    hipLaunchKernelGGL(k_fft_rows_inv<false>, dim3((n / 2 + RP - 1) / RP, nb), block,
                       bpre ? lds_inv : lds, s, spec, n, RP, pc->fp, pc->d_tw, base, out, bpre);
  }
  CT_TRY_HIP(hipGetLastError());
  return CT_OK;
}

bool fft_factor(int L, FftPlan *fp) {
  fp->L = L;
  fp->npass = 0;
  int m = L, twos = 0;
  while (m % 2 == 0) {
    m /= 2;
    ++twos;
  }
  // powers of two as radix 8 passes, the remainder as one radix-4 or -2 pass
  // (or, for 2^(3k+1) with k >= 1, two radix-4 passes instead of 8 and 2)
  int eights = twos / 3, rest = twos % 3;
  if (rest == 1 && eights > 0) {
    --eights;
    rest = 4;  // 2^4 = 4 x 4
  }
  for (int i = 0; i < eights; ++i) fp->radix[fp->npass++] = 8;
  if (rest == 4) {
    fp->radix[fp->npass++] = 4;
    fp->radix[fp->npass++] = 4;
  } else if (rest == 2) {
    fp->radix[fp->npass++] = 4;
  } else if (rest == 1) {
    fp->radix[fp->npass++] = 2;
  }
  while (m % 3 == 0) {
    fp->radix[fp->npass++] = 3;
    m /= 3;
    if (fp->npass > 16) return false;
  }
  fp->code = 0;
  for (int i = 0; i < fp->npass; ++i) fp->code |= (uint64_t)fp->radix[i] << (4 * i);
  // quads for power-of-two lengths where one problem's row block leaves
  // lanes idle in a radix-8 pass (L <= 512)
  fp->quad8 = (L & (L - 1)) == 0 && rows_per_block(L) * (L / 8) < kFftThreads ? 1 : 0;
  return m == 1 && fp->npass <= 16;
}

}  // namespace ctpd
