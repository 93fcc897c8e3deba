// The conjugate-gradient pieces of ADMM's u-step (thesis §4.6): FP64 dot
// products into device scalars, and the two vector updates that read their
// step lengths from those scalars, so that an ADMM iteration needs no host
// round trip (and captures into a graph).
#include "common.hpp"

namespace ctpd {

constexpr int kDotThreads = 256;
constexpr int kDotBlocks = 512;

// partials[block] = sum over the block's grid-stride share of x[t] y[t] (FP64)
__global__ __launch_bounds__(kDotThreads) void k_dot(const float *__restrict__ x,
                                                     const float *__restrict__ y, int64_t count,
                                                     double *__restrict__ partials) {
  double v = 0.0;
  for (int64_t t = (int64_t)blockIdx.x * kDotThreads + threadIdx.x; t < count;
       t += (int64_t)gridDim.x * kDotThreads)
    v = fma((double)x[t], (double)y[t], v);
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  __shared__ double sh[kDotThreads / 64];
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double acc = sh[0];
    for (int w = 1; w < kDotThreads / 64; ++w) acc += sh[w];
    partials[blockIdx.x] = acc;
  }
}

// out[0] = sum of the partials, in a fixed order (deterministic)
__global__ __launch_bounds__(kDotThreads) void k_dot_finalize(const double *__restrict__ partials,
                                                              int count, double *__restrict__ out) {
  double v = 0.0;
  for (int t = threadIdx.x; t < count; t += kDotThreads) v += partials[t];
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  __shared__ double sh[kDotThreads / 64];
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double acc = sh[0];
    for (int w = 1; w < kDotThreads / 64; ++w) acc += sh[w];
    out[0] = acc;
  }
}

// alpha = r.z / p.Hp (0 when p.Hp = 0, a zero residual); u += alpha p; r -= alpha Hp
__global__ void k_cg_update(int64_t count, const double *__restrict__ rz,
                            const double *__restrict__ pHp, const float *__restrict__ p,
                            const float *__restrict__ Hp, float *__restrict__ u,
                            float *__restrict__ r) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= count) return;
  const double d = pHp[0];
  const float a = d > 0.0 ? (float)(rz[0] / d) : 0.f;
  u[t] = fmaf(a, p[t], u[t]);
  r[t] = fmaf(-a, Hp[t], r[t]);
}

// p = z + beta p with beta = rz_new / rz_old (0 when rz_old = 0); p = z when
// rz_old is null (the first direction)
__global__ void k_cg_dir(int64_t count, const double *__restrict__ rz_new,
                         const double *__restrict__ rz_old, const float *__restrict__ z,
                         float *__restrict__ p) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= count) return;
  if (rz_old == nullptr) {
    p[t] = z[t];
    return;
  }
  const double o = rz_old[0];
  const float b = o > 0.0 ? (float)(rz_new[0] / o) : 0.f;
  p[t] = fmaf(b, p[t], z[t]);
}

size_t dot_partials_needed() { return kDotBlocks; }

int launch_dot(const float *x, const float *y, int64_t count, double *partials, double *out,
               hipStream_t s) {
  hipLaunchKernelGGL(k_dot, dim3(kDotBlocks), dim3(kDotThreads), 0, s, x, y, count, partials);
  CT_TRY_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_dot_finalize, dim3(1), dim3(kDotThreads), 0, s, partials, kDotBlocks, out);
  CT_TRY_HIP(hipGetLastError());
  return CT_OK;
}

int launch_cg_update(int64_t count, const double *rz, const double *pHp, const float *p,
                     const float *Hp, float *u, float *r, hipStream_t s) {
  hipLaunchKernelGGL(k_cg_update, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, count,
                     rz, pHp, p, Hp, u, r);
  CT_TRY_HIP(hipGetLastError());
  return CT_OK;
}

int launch_cg_dir(int64_t count, const double *rz_new, const double *rz_old, const float *z,
                  float *p, hipStream_t s) {
  hipLaunchKernelGGL(k_cg_dir, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, count,
                     rz_new, rz_old, z, p);
  CT_TRY_HIP(hipGetLastError());
  return CT_OK;
}

}  // namespace ctpd
