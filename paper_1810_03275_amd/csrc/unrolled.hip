// Reverse sweep of K unrolled PDRQS1 iterations (thesis §4.4): the pointwise
// parts of the chain rule through one iteration, for nb problems at once.
//
// One iteration from (u, vb1, vb2), A = R_h/beta, b = u0/beta, rho = lambda~/tau:
//   u'   = u + M^{-1}(-sigma A^*(vb1 + sigma A u) + sigma tau div(vb2 + sigma tau nabla u))
//   q1   = vb1 + 2 sigma A u',      y1 = P1(q1; b),   vb1' = y1 - sigma A u'
//   q2   = vb2 + 2 sigma tau nabla u',  w = P2(q2; rho),  vb2' = w - sigma tau nabla u'
// with P1 = (q - sigma b)/(1 + sigma) off D0, min(q - sigma C~, 0) on D0, and
// P2 the pixelwise projection onto the ball of radius rho.  Given the
// adjoints (U, V1, V2) of (u', vb1', vb2') and a deferred sinogram term P
// (A^* P belongs to U), one reverse step is
//   Q1 = P1'(q1) V1,  bbar += dP1/db V1,  P += -sigma V1 + 2 sigma Q1     (k_sino_reverse)
//   Q2 = P2'(q2)^T V2, rhobar += dP2/drho . V2, G = sigma tau (2 Q2 - V2)   (k_tv_reverse)
//   Utot = U + A^* P - div G                                            (R_h^* epilogue)
//   X = M^{-1} Utot                                                     (FFT pair)
//   S1 = -sigma A X:  V1 <- Q1 + S1,  P <- sigma S1                     (R_h epilogue, mode 3)
//   S2 = -sigma tau nabla X:  V2 <- Q2 + S2,  U <- Utot - sigma tau div S2  (k_img_tail)
#include "common.hpp"

namespace ctpd {

constexpr int kRevThreads = 256;

__global__ void k_sino_reverse(int N, int M, float sigma, const float *__restrict__ V1,
                               const float *__restrict__ q1, const float *__restrict__ target,
                               const uint32_t *__restrict__ mask, float *__restrict__ P,
                               float *__restrict__ Q1, float *__restrict__ bbar) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const int l = blockIdx.y;
  if (k >= M) return;
  const size_t NM = (size_t)N * M;
  const int MW = (M + 31) >> 5;
  const size_t o = blockIdx.z * NM + (size_t)l * M + k;
  const bool on = mask != nullptr &&
                  ((mask[blockIdx.z * (size_t)N * MW + (size_t)l * MW + (k >> 5)] >> (k & 31)) & 1u);
  const float v = V1[o];
  const float inv1 = 1.f / (1.f + sigma);
  // on D0 the resolvent is min(q - sigma C~, 0): slope 1 below the kink, 0 above
  const float d1 = on ? ((q1[o] - sigma * target[o] < 0.f) ? 1.f : 0.f) : inv1;
  const float Q = d1 * v;
  Q1[o] = Q;
  if (!on) bbar[o] = fmaf(-sigma * inv1, v, bbar[o]);
  P[o] += sigma * (2.f * Q - v);
}

__global__ __launch_bounds__(kRevThreads) void k_tv_reverse(
    int n, float st, float rho, const float *__restrict__ V2, const float *__restrict__ q2,
    float *__restrict__ Q2, float *__restrict__ G, double *__restrict__ partials) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  const size_t nn = (size_t)n * n;
  double part = 0.0;
  if (i < n) {
    const size_t o = blockIdx.z * 2 * nn + (size_t)j * n + i;
    const float w1 = V2[o], w2 = V2[o + nn];
    const float a = q2[o], b = q2[o + nn];
    const float nq = sqrtf(a * a + b * b);
    float r1 = w1, r2 = w2;
    if (nq > rho) {
      // (rho/|q|)(I - qhat qhat^T) w, and d/drho of rho qhat is qhat
      const float h1 = a / nq, h2 = b / nq;
      const float dot = h1 * w1 + h2 * w2;
      const float sc = rho / nq;
      r1 = sc * (w1 - h1 * dot);
      r2 = sc * (w2 - h2 * dot);
      part = (double)dot;
    }
    Q2[o] = r1;
    Q2[o + nn] = r2;
    G[o] = st * (2.f * r1 - w1);
    G[o + nn] = st * (2.f * r2 - w2);
  }
  // block sum in FP64, fixed order
  __shared__ double sh[kRevThreads / 64];
  for (int off = 32; off > 0; off >>= 1) part += __shfl_xor(part, off, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = part;
  __syncthreads();
  if (threadIdx.x == 0) {
    double acc = sh[0];
    for (int w = 1; w < kRevThreads / 64; ++w) acc += sh[w];
    partials[(size_t)blockIdx.z * gridDim.x * gridDim.y + (size_t)blockIdx.y * gridDim.x +
             blockIdx.x] = acc;
  }
}

// acc[b] += sum of problem b's partials (one block per problem, fixed order).
__global__ __launch_bounds__(kRevThreads) void k_partials_add(const double *__restrict__ partials,
                                                              int count, double *__restrict__ acc) {
  const double *p = partials + (size_t)blockIdx.x * count;
  double v = 0.0;
  for (int t = threadIdx.x; t < count; t += kRevThreads) v += p[t];
  __shared__ double sh[kRevThreads / 64];
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = sh[0];
    for (int w = 1; w < kRevThreads / 64; ++w) s += sh[w];
    acc[blockIdx.x] += s;
  }
}

__global__ void k_img_tail(int n, float st, float inv_h, const float *__restrict__ X,
                           const float *__restrict__ Q2, const float *__restrict__ Utot,
                           float *__restrict__ Uout, float *__restrict__ V2out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (i >= n) return;
  const size_t nn = (size_t)n * n;
  const size_t o = (size_t)j * n + i;
  X += blockIdx.z * nn;
  Utot += blockIdx.z * nn;
  Uout += blockIdx.z * nn;
  Q2 += blockIdx.z * 2 * nn;
  V2out += blockIdx.z * 2 * nn;
  const float x = X[o];
  // S2 = -sigma tau nabla X at (i, j), (i-1, j) and (i, j-1)
  const float s1 = (i < n - 1) ? -st * (X[o + 1] - x) * inv_h : 0.f;
  const float s2 = (j < n - 1) ? -st * (X[o + n] - x) * inv_h : 0.f;
  const float s1l = (i > 0) ? -st * (x - X[o - 1]) * inv_h : 0.f;
  const float s2d = (j > 0) ? -st * (x - X[o - n]) * inv_h : 0.f;
  V2out[o] = Q2[o] + s1;
  V2out[o + nn] = Q2[o + nn] + s2;
  // div S2 with the same boundary rule as div_h
  const float dv = ((i < n - 1 ? s1 : 0.f) - s1l + (j < n - 1 ? s2 : 0.f) - s2d) * inv_h;
  Uout[o] = Utot[o] - st * dv;
}

int launch_sino_reverse(int N, int M, int nb, float sigma, const float *V1, const float *q1,
                        const float *target, const uint32_t *mask, float *P, float *Q1,
                        float *bbar, hipStream_t s) {
  hipLaunchKernelGGL(k_sino_reverse, dim3((M + 255) / 256, N, nb), dim3(256), 0, s, N, M, sigma,
                     V1, q1, target, mask, P, Q1, bbar);
  CT_TRY_HIP(hipGetLastError());
  return CT_OK;
}

size_t tv_reverse_partials(int n, int nb) {
  return (size_t)((n + kRevThreads - 1) / kRevThreads) * n * nb;
}

int launch_tv_reverse(int n, int nb, float sigtau, float rho, const float *V2, const float *q2,
                      float *Q2, float *G, double *partials, double *acc, hipStream_t s) {
  const int bx = (n + kRevThreads - 1) / kRevThreads;
  hipLaunchKernelGGL(k_tv_reverse, dim3(bx, n, nb), dim3(kRevThreads), 0, s, n, sigtau, rho, V2,
                     q2, Q2, G, partials);
  CT_TRY_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_partials_add, dim3(nb), dim3(kRevThreads), 0, s, partials, bx * n, acc);
  CT_TRY_HIP(hipGetLastError());
  return CT_OK;
}

int launch_img_tail(int n, int nb, float sigtau, float inv_h, const float *X, const float *Q2,
                    const float *Utot, float *Uout, float *V2out, hipStream_t s) {
  hipLaunchKernelGGL(k_img_tail, dim3((n + 255) / 256, n, nb), dim3(256), 0, s, n, sigtau, inv_h,
                     X, Q2, Utot, Uout, V2out);
  CT_TRY_HIP(hipGetLastError());
  return CT_OK;
}

}  // namespace ctpd
