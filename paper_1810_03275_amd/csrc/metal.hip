// Metal-trace estimate from a reconstruction (thesis, results chapter, real
// metal artifacts): pixels above a threshold, dilated by a disk of radius r,
// carried to the sinogram by R_h; D0 holds the bins the projection reaches
// with more than kappa, and optionally C = c0 u0 on D0.
#include "common.hpp"

namespace ctpd {

constexpr int kDilTile = 32;  // pixels per side of a workgroup's tile
constexpr int kDilThreads = 256;

// chi[j][i] = 1 iff some pixel (i + a, j + b) of the image with
// a^2 + b^2 <= r^2 has u > thr.  The tile's marks plus a halo of r pixels
// are staged in LDS as bytes.
__global__ __launch_bounds__(kDilThreads) void k_mark_dilate(int n, const float *__restrict__ u,
                                                             float thr, int r,
                                                             float *__restrict__ chi) {
  __shared__ unsigned char m[(kDilTile + 2 * kDilMaxRadius) * (kDilTile + 2 * kDilMaxRadius)];
  const int W = kDilTile + 2 * r;
  const int i0 = blockIdx.x * kDilTile - r, j0 = blockIdx.y * kDilTile - r;
  for (int t = threadIdx.x; t < W * W; t += kDilThreads) {
    const int b = t / W, a = t - b * W;
    const int i = i0 + a, j = j0 + b;
    m[t] = (i >= 0 && i < n && j >= 0 && j < n && u[(size_t)j * n + i] > thr) ? 1 : 0;
  }
  __syncthreads();
  for (int t = threadIdx.x; t < kDilTile * kDilTile; t += kDilThreads) {
    const int b = t / kDilTile, a = t - b * kDilTile;
    const int i = blockIdx.x * kDilTile + a, j = blockIdx.y * kDilTile + b;
    if (i >= n || j >= n) continue;
    bool hit = false;
    for (int db = -r; db <= r && !hit; ++db) {
      const unsigned char *row = m + (b + r + db) * W + (a + r);
      for (int da = -r; da <= r; ++da) {
        if (da * da + db * db <= r * r && row[da]) {
          hit = true;
          break;
        }
      }
    }
    chi[(size_t)j * n + i] = hit ? 1.f : 0.f;
  }
}

// D0 bit k & 31 of word k >> 5 of row l: proj[l][k] > kappa (bins >= M are 0);
// bound[l][k] = c0 u0[l][k] on D0, 0 elsewhere (when bound is given).  One
// thread per bin of the padded row, words assembled with a wave ballot.
__global__ __launch_bounds__(256) void k_trace_mask(int M, int MW, const float *__restrict__ proj,
                                                    float kappa, uint32_t *__restrict__ mask,
                                                    const float *__restrict__ u0, float c0,
                                                    float *__restrict__ bound) {
  const int l = blockIdx.y;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;  // < 32 MW rounded up to 256
  const size_t o = (size_t)l * M + k;
  const bool on = k < M && proj[o] > kappa;
  const uint64_t bits = __ballot(on);
  const int lane = threadIdx.x & 63;
  const int w = k >> 5;
  if ((lane & 31) == 0 && w < MW) mask[(size_t)l * MW + w] = (uint32_t)(bits >> lane);
  if (bound != nullptr && k < M) bound[o] = on ? c0 * u0[o] : 0.f;
}

int launch_d0_estimate(const ct_plan *p, const float *u, float thr, int r, float kappa,
                       float *chi, float *proj, uint32_t *mask, const float *u0, float c0,
                       float *bound, hipStream_t s) {
  const int n = p->g.n, N = p->g.n_angles, M = p->g.n_bins;
  const int MW = (M + 31) / 32;
  const dim3 tiles((n + kDilTile - 1) / kDilTile, (n + kDilTile - 1) / kDilTile);
  hipLaunchKernelGGL(k_mark_dilate, tiles, dim3(kDilThreads), 0, s, n, u, thr, r, chi);
  CT_TRY_HIP(hipGetLastError());
  CT_TRY(launch_radon_fwd(p, chi, proj, s));
  hipLaunchKernelGGL(k_trace_mask, dim3((32 * MW + 255) / 256, N), dim3(256), 0, s, M, MW, proj,
                     kappa, mask, u0, c0, bound);
  CT_TRY_HIP(hipGetLastError());
  return CT_OK;
}

}  // namespace ctpd
