// Stencil, pointwise and reduction kernels of PDRQS1 (thesis §3.1, §3.3,
// §4.4) and the FP64 record.  All HBM-bound; one thread per element.
#include <cmath>

#include "common.hpp"
#include "tv_update.hpp"

namespace ctpd {

__device__ inline bool mask_bit(const uint32_t *__restrict__ mask, int MW, int l, int k) {
  return mask != nullptr && ((mask[(size_t)l * MW + (k >> 5)] >> (k & 31)) & 1u);
}

// ---------------------------------------------------------------------------
// nabla_h (forward differences, zero on the far edge) and div_h = -nabla_h^T.
__global__ void k_grad(int n, float inv_h, const float *__restrict__ u, float *__restrict__ p) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (i >= n) return;
  const size_t o = (size_t)j * n + i;
  const float c = u[o];
  p[o] = (i < n - 1) ? (u[o + 1] - c) * inv_h : 0.f;
  p[o + (size_t)n * n] = (j < n - 1) ? (u[o + n] - c) * inv_h : 0.f;
}

__global__ void k_div(int n, float inv_h, const float *__restrict__ p, float *__restrict__ d) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (i >= n) return;
  const size_t o = (size_t)j * n + i;
  const float *p1 = p, *p2 = p + (size_t)n * n;
  const float d1 = (i < n - 1 ? p1[o] : 0.f) - (i > 0 ? p1[o - 1] : 0.f);
  const float d2 = (j < n - 1 ? p2[o] : 0.f) - (j > 0 ? p2[o - n] : 0.f);
  d[o] = (d1 + d2) * inv_h;
}

__global__ void k_tv_project(int64_t count, const float *__restrict__ q, float radius,
                             float *__restrict__ w) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= count) return;
  float w1, w2;
  ball_project(q[t], q[t + count], radius, w1, w2);
  w[t] = w1;
  w[t + count] = w2;
}

// PDRQS1 gradient-side update (§4.4), one thread per pixel (tv_update_px).
__global__ void k_tv_update(TvArgs a) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  tv_update_px(a, i, blockIdx.y, blockIdx.z);
}

// ---------------------------------------------------------------------------
// Sinogram resolvent (§3.3 / §4.4): off D0 (q - s u0)/(1+s), on D0 min(q - s C, 0).
__global__ void k_prox_sino(int N, int M, const float *__restrict__ q, float step,
                            const float *__restrict__ u0, const float *__restrict__ bound,
                            const uint32_t *__restrict__ mask, float *__restrict__ y) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const int l = blockIdx.y;
  if (k >= M) return;
  const size_t o = (size_t)l * M + k;
  const int MW = (M + 31) >> 5;
  const float qq = q[o];
  y[o] = mask_bit(mask, MW, l, k) ? fminf(qq - step * bound[o], 0.f)
                                  : (qq - step * u0[o]) / (1.f + step);
}

// PDRQS1 sinogram-side update (§4.4) from the raw projection R_h u:
// r = R_h u / beta, v1 = vb1 + sigma r, y1 = prox(2 v1 - vb1), vb1 <- vb1 + y1 - v1,
// s1 = vb1 + sigma r.  target holds b = u0/beta off D0 and C/beta on D0.
// mode 1: only s1 = vb1 + sigma r.  mode 2: also store y1 and r.
__global__ void k_sino_update(int N, int M, const float *__restrict__ rraw, float inv_beta,
                              float sigma, const float *__restrict__ target,
                              const uint32_t *__restrict__ mask, float *__restrict__ vb1,
                              float *__restrict__ s1, float *__restrict__ y1out,
                              float *__restrict__ rout, int mode) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const int l = blockIdx.y;
  if (k >= M) return;
  const size_t o = (size_t)l * M + k;
  const float r = rraw[o] * inv_beta;
  const float vb = vb1[o];
  if (mode == 1) {
    s1[o] = fmaf(sigma, r, vb);
    return;
  }
  const int MW = (M + 31) >> 5;
  const float v1 = fmaf(sigma, r, vb);
  const float q = 2.f * v1 - vb;
  const float tg = target[o];
  const float y = mask_bit(mask, MW, l, k) ? fminf(q - sigma * tg, 0.f)
                                           : (q - sigma * tg) / (1.f + sigma);
  const float nb = vb + y - v1;
  vb1[o] = nb;
  s1[o] = fmaf(sigma, r, nb);
  if (mode == 2) {
    y1out[o] = y;
    rout[o] = r;
  }
}

__global__ void k_build_target(int N, int M, const float *__restrict__ u0,
                               const float *__restrict__ bound, float bscalar,
                               const uint32_t *__restrict__ mask, float inv_beta,
                               float *__restrict__ target) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const int l = blockIdx.y;
  if (k >= M) return;
  const size_t o = (size_t)l * M + k;
  const int MW = (M + 31) >> 5;
  const float v = mask_bit(mask, MW, l, k) ? (bound ? bound[o] : bscalar) : u0[o];
  target[o] = v * inv_beta;
}

// ---------------------------------------------------------------------------
// FP64 reductions: a fixed grid of kRedBlocks blocks writes per-block partials,
// one block combines them in a fixed order (deterministic).
constexpr int kRedBlocks = 512;
constexpr int kRedThreads = 256;

__device__ inline double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}
__device__ inline double wave_max(double v) {
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}

// Block-level combine of NV values (bit v of maxmask: max instead of sum).
template <int NV>
__device__ void block_reduce_store(double (&v)[NV], unsigned maxmask, double *dst) {
  __shared__ double sh[kRedThreads / 64][NV];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
  for (int q = 0; q < NV; ++q) v[q] = ((maxmask >> q) & 1u) ? wave_max(v[q]) : wave_sum(v[q]);
  if (lane == 0) {
#pragma unroll
    for (int q = 0; q < NV; ++q) sh[wave][q] = v[q];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      double acc = sh[0][q];
      for (int w = 1; w < kRedThreads / 64; ++w)
        acc = ((maxmask >> q) & 1u) ? fmax(acc, sh[w][q]) : acc + sh[w][q];
      dst[q] = acc;
    }
  }
}

template <int NV>
__global__ void k_finalize(const double *__restrict__ partials, int nblocks, unsigned maxmask,
                           unsigned sqrtmask, double *__restrict__ out) {
  double v[NV];
#pragma unroll
  for (int q = 0; q < NV; ++q) v[q] = ((maxmask >> q) & 1u) ? 0.0 : 0.0;
  for (int b = threadIdx.x; b < nblocks; b += blockDim.x) {
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      const double x = partials[(size_t)b * NV + q];
      v[q] = ((maxmask >> q) & 1u) ? fmax(v[q], x) : v[q] + x;
    }
  }
  __shared__ double res[NV];
  block_reduce_store<NV>(v, maxmask, res);
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < NV; ++q) out[q] = ((sqrtmask >> q) & 1u) ? sqrt(res[q]) : res[q];
  }
}

__global__ void k_sumsq(const float *__restrict__ x, int64_t count, double *partials) {
  double v[1] = {0.0};
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < count;
       t += (int64_t)gridDim.x * blockDim.x) {
    const double a = x[t];
    v[0] = fma(a, a, v[0]);
  }
  block_reduce_store<1>(v, 0u, partials + blockIdx.x);
}

__global__ void k_scale_by_inv(const float *__restrict__ x, int64_t count,
                               const double *__restrict__ norm, float *__restrict__ y) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= count) return;
  const double s = 1.0 / norm[0];
  y[t] = (float)((double)x[t] * s);
}

__global__ void k_nonfinite(const float *__restrict__ x, int64_t count, int *flag) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= count) return;
  if (!isfinite(x[t])) atomicOr(flag, 1);
}

__global__ void k_sino_gap(int N, int M, const float *__restrict__ r, const float *__restrict__ y1,
                           const float *__restrict__ target, const uint32_t *__restrict__ mask,
                           double *partials) {
  double v[3] = {0.0, 0.0, 0.0};
  const int MW = (M + 31) >> 5;
  const int64_t count = (int64_t)N * M;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < count;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int l = (int)(t / M), k = (int)(t - (int64_t)l * M);
    const double rr = r[t], yy = y1[t], tg = target[t];
    if (mask_bit(mask, MW, l, k)) {
      v[1] = fma(yy, tg, v[1]);
      v[2] = fmax(v[2], tg - rr);
    } else {
      const double d = rr - tg;
      v[0] = fma(0.5 * d, d, v[0]);
      v[1] += yy * (0.5 * yy + tg);
    }
  }
  block_reduce_store<3>(v, 4u, partials + (size_t)blockIdx.x * 3);
}

__global__ void k_img_gap(int n, float inv_h, const float *__restrict__ u,
                          const float *__restrict__ uprev, const float *__restrict__ z,
                          double *partials) {
  double v[3] = {0.0, 0.0, 0.0};
  const int64_t count = (int64_t)n * n;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < count;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int j = (int)(t / n), i = (int)(t - (int64_t)j * n);
    const double c = u[t];
    const double g1 = (i < n - 1) ? ((double)u[t + 1] - c) * inv_h : 0.0;
    const double g2 = (j < n - 1) ? ((double)u[t + n] - c) * inv_h : 0.0;
    v[0] += sqrt(g1 * g1 + g2 * g2);
    const double du = c - (double)uprev[t];
    v[1] = fma(du, du, v[1]);
    const double zz = z[t];
    v[2] = fma(zz, zz, v[2]);
  }
  block_reduce_store<3>(v, 0u, partials + (size_t)blockIdx.x * 3);
}

// ---------------------------------------------------------------------------
// launchers

static dim3 row_grid(int len, int rows) { return dim3((len + 255) / 256, rows); }

int launch_grad(int n, float inv_h, const float *u, float *p, hipStream_t s) {
  hipLaunchKernelGGL(k_grad, row_grid(n, n), dim3(256), 0, s, n, inv_h, u, p);
  CT_TRY_HIP(hipGetLastError());
  return CT_OK;
}

int launch_div(int n, float inv_h, const float *p, float *d, hipStream_t s) {
  hipLaunchKernelGGL(k_div, row_grid(n, n), dim3(256), 0, s, n, inv_h, p, d);
  CT_TRY_HIP(hipGetLastError());
  return CT_OK;
}

int launch_tv_project(int n, const float *q, float radius, float *w, hipStream_t s) {
  const int64_t count = (int64_t)n * n;
  hipLaunchKernelGGL(k_tv_project, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, count,
                     q, radius, w);
  CT_TRY_HIP(hipGetLastError());
  return CT_OK;
}

int launch_tv_update(int n, float inv_h, const float *u, float sigtau, float radius, float *vb2,
                     float *s2, float *wout, int mode, hipStream_t s, int nb, float *q2out,
                     float *ubar) {
  dim3 grid = row_grid(n, n);
  grid.z = nb;
  TvArgs a;
  a.n = n;
  a.inv_h = inv_h;
  a.u = u;
  a.st = sigtau;
  a.radius = radius;
  a.vb2 = vb2;
  a.s2 = s2;
  a.wout = wout;
  a.mode = mode;
  a.q2out = q2out;
  a.ubar = ubar;
  hipLaunchKernelGGL(k_tv_update, grid, dim3(256), 0, s, a);
  CT_TRY_HIP(hipGetLastError());
  return CT_OK;
}

__global__ void k_axpy(int64_t count, const float *__restrict__ base, float a,
                       const float *__restrict__ x, float *__restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < count) out[t] = fmaf(a, x[t], base[t]);
}

// Objective terms of (C_h): sinogram part (fit off D0, violation on D0) and
// the total variation, in FP64 (one pass each, fixed-order reductions).
__global__ void k_obj_sino(int N, int M, const float *__restrict__ r, const float *__restrict__ u0,
                           const float *__restrict__ bound, float bscalar,
                           const uint32_t *__restrict__ mask, double *partials) {
  double v[2] = {0.0, 0.0};
  const int MW = (M + 31) >> 5;
  const int64_t count = (int64_t)N * M;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < count;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int l = (int)(t / M), k = (int)(t - (int64_t)l * M);
    const double rr = r[t];
    if (mask_bit(mask, MW, l, k)) {
      const double cb = bound ? (double)bound[t] : (double)bscalar;
      v[1] = fmax(v[1], cb - rr);
    } else {
      const double d = rr - u0[t];
      v[0] = fma(0.5 * d, d, v[0]);
    }
  }
  block_reduce_store<2>(v, 2u, partials + (size_t)blockIdx.x * 2);
}

__global__ void k_obj_tv(int n, float inv_h, const float *__restrict__ u, double *partials) {
  double v[1] = {0.0};
  const int64_t count = (int64_t)n * n;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < count;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int j = (int)(t / n), i = (int)(t - (int64_t)j * n);
    const double c = u[t];
    const double g1 = (i < n - 1) ? (u[t + 1] - c) * inv_h : 0.0;
    const double g2 = (j < n - 1) ? (u[t + n] - c) * inv_h : 0.0;
    v[0] += sqrt(g1 * g1 + g2 * g2);
  }
  block_reduce_store<1>(v, 0u, partials + blockIdx.x);
}

int launch_axpy(int64_t count, const float *base, float a, const float *x, float *out,
                hipStream_t s) {
  hipLaunchKernelGGL(k_axpy, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, count, base,
                     a, x, out);
  CT_TRY_HIP(hipGetLastError());
  return CT_OK;
}

int launch_objective(int N, int M, const float *r, const float *u0, const float *bound,
                     float bscalar, const uint32_t *mask, int n, float inv_h, const float *u,
                     double *partials, int cap, double *out, hipStream_t s) {
  if (cap < kRedBlocks * 2) {
    set_error("objective: reduction buffer too small");
    return CT_E_INVALID;
  }
  hipLaunchKernelGGL(k_obj_sino, dim3(kRedBlocks), dim3(kRedThreads), 0, s, N, M, r, u0, bound,
                     bscalar, mask, partials);
  hipLaunchKernelGGL(k_finalize<2>, dim3(1), dim3(kRedThreads), 0, s, partials, kRedBlocks, 2u,
                     0u, out);
  hipLaunchKernelGGL(k_obj_tv, dim3(kRedBlocks), dim3(kRedThreads), 0, s, n, inv_h, u, partials);
  hipLaunchKernelGGL(k_finalize<1>, dim3(1), dim3(kRedThreads), 0, s, partials, kRedBlocks, 0u,
                     0u, out + 2);
  CT_TRY_HIP(hipGetLastError());
  return CT_OK;
}

int launch_prox_sino(int N, int M, const float *q, float step, const float *u0,
                     const float *bound, const uint32_t *mask, float *y, hipStream_t s) {
  hipLaunchKernelGGL(k_prox_sino, row_grid(M, N), dim3(256), 0, s, N, M, q, step, u0, bound,
                     mask, y);
  CT_TRY_HIP(hipGetLastError());
  return CT_OK;
}

int launch_sino_update(int N, int M, const float *rraw, float inv_beta, float sigma,
                       const float *target, const uint32_t *mask, float *vb1, float *s1,
                       float *y1, float *rout, int mode, hipStream_t s) {
  hipLaunchKernelGGL(k_sino_update, row_grid(M, N), dim3(256), 0, s, N, M, rraw, inv_beta,
                     sigma, target, mask, vb1, s1, y1, rout, mode);
  CT_TRY_HIP(hipGetLastError());
  return CT_OK;
}

int launch_build_target(int N, int M, const float *u0, const float *bound, float bscalar,
                        const uint32_t *mask, float inv_beta, float *target, hipStream_t s) {
  hipLaunchKernelGGL(k_build_target, row_grid(M, N), dim3(256), 0, s, N, M, u0, bound, bscalar,
                     mask, inv_beta, target);
  CT_TRY_HIP(hipGetLastError());
  return CT_OK;
}

int reduction_partials_needed() { return kRedBlocks * 3; }

int launch_norm2(const float *x, int64_t count, double *partials, int cap, double *out,
                 hipStream_t s) {
  if (cap < kRedBlocks) {
    set_error("reduction workspace too small");
    return CT_E_INVALID;
  }
  hipLaunchKernelGGL(k_sumsq, dim3(kRedBlocks), dim3(kRedThreads), 0, s, x, count, partials);
  CT_TRY_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_finalize<1>, dim3(1), dim3(kRedThreads), 0, s, partials, kRedBlocks, 0u,
                     1u, out);
  CT_TRY_HIP(hipGetLastError());
  return CT_OK;
}

int launch_scale_by_inv(const float *x, int64_t count, const double *norm, float *y,
                        hipStream_t s) {
  hipLaunchKernelGGL(k_scale_by_inv, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, x,
                     count, norm, y);
  CT_TRY_HIP(hipGetLastError());
  return CT_OK;
}

int launch_nonfinite(const float *x, int64_t count, int *flag, hipStream_t s) {
  if (count <= 0) return CT_OK;
  hipLaunchKernelGGL(k_nonfinite, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, x,
                     count, flag);
  CT_TRY_HIP(hipGetLastError());
  return CT_OK;
}

int launch_sino_gap(int N, int M, const float *r, const float *y1, const float *target,
                    const uint32_t *mask, double *partials, int cap, double *out,
                    hipStream_t s) {
  if (cap < kRedBlocks * 3) {
    set_error("reduction workspace too small");
    return CT_E_INVALID;
  }
  hipLaunchKernelGGL(k_sino_gap, dim3(kRedBlocks), dim3(kRedThreads), 0, s, N, M, r, y1, target,
                     mask, partials);
  CT_TRY_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_finalize<3>, dim3(1), dim3(kRedThreads), 0, s, partials, kRedBlocks, 4u,
                     0u, out);
  CT_TRY_HIP(hipGetLastError());
  return CT_OK;
}

int launch_img_gap(int n, float inv_h, const float *u, const float *uprev, const float *z,
                   double *partials, int cap, double *out, hipStream_t s) {
  if (cap < kRedBlocks * 3) {
    set_error("reduction workspace too small");
    return CT_E_INVALID;
  }
  hipLaunchKernelGGL(k_img_gap, dim3(kRedBlocks), dim3(kRedThreads), 0, s, n, inv_h, u, uprev, z,
                     partials);
  CT_TRY_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_finalize<3>, dim3(1), dim3(kRedThreads), 0, s, partials, kRedBlocks, 0u,
                     0u, out);
  CT_TRY_HIP(hipGetLastError());
  return CT_OK;
}

}  // namespace ctpd
