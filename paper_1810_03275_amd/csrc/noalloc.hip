// ct_power_norm_noalloc: the power iteration of ct_power_norm (§5.1: beta =
// ||R_h|| by power steps on R_h^* R_h) for callers that cannot allocate
// device memory.  Its work image, sinogram and FP64 reduction partials live
// in one file-scope device array instead of the plan's scratch.
#include <mutex>

#include "common.hpp"

namespace ctpd {

namespace {

// The work image (n^2 floats), the sinogram (N M floats) and the reduction
// partials (FP64, 256-byte aligned) of one call.
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;  // 64 MiB

__device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void *g_scratch_ptr[kMaxDevices] = {};

// The device address of `scratch` on the current device, looked up once per
// device (each device holds its own copy of the array).
int scratch_on_current_device(void **out) {
  int dev = 0;
  CT_TRY_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) {
    set_error("ct_power_norm_noalloc: device index out of range");
    return CT_E_UNSUPPORTED;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    CT_TRY_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return CT_OK;
}

// The start image used when the caller gives none (the same smooth,
// non-symmetric, non-zero-mean image as ct_power_norm's).
__global__ void k_default_start(int n, float *x) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (i >= n) return;
  x[(size_t)j * n + i] =
      (float)(1.0 + 0.5 * sin(0.37 * i + 1.13 * j) + 0.25 * cos(0.071 * i * j + 0.3));
}

}  // namespace

// Looks up the array on the current device ahead of the entry point's first
// call there (plan creation calls this), so that the runtime's one-time
// loading of the array happens at set-up, not inside a no-allocation call.
int noalloc_prepare_device() {
  void *ptr = nullptr;
  return scratch_on_current_device(&ptr);
}

}  // namespace ctpd

using namespace ctpd;

extern "C" int ct_power_norm_noalloc(const ct_plan *p, int32_t iters, const float *x0,
                                     double *out, ct_stream s) {
  clear_error();
  if (!p || !out || iters < 1) {
    set_error("ct_power_norm_noalloc: invalid argument");
    return CT_E_INVALID;
  }
  const int n = p->g.n;
  const size_t nn = (size_t)n * n, NM = (size_t)p->g.n_angles * p->g.n_bins;
  const size_t img_bytes = nn * sizeof(float), sino_bytes = NM * sizeof(float);
  const size_t red_off = (img_bytes + sino_bytes + 255) & ~size_t(255);
  const int red_cap = reduction_partials_needed() + 16;
  const size_t need = red_off + sizeof(double) * (size_t)red_cap;
  if (need > kNoAllocScratchBytes) {
    set_error("ct_power_norm_noalloc: the image and sinogram need " + std::to_string(need) +
              " bytes of scratch; the library's array holds " +
              std::to_string(kNoAllocScratchBytes) + " (n^2 + N M <= about 16.7 million)");
    return CT_E_INVALID;
  }
  void *base = nullptr;
  CT_TRY(scratch_on_current_device(&base));
  unsigned char *b = static_cast<unsigned char *>(base);
  float *x = reinterpret_cast<float *>(b);
  float *sino = reinterpret_cast<float *>(b + img_bytes);
  double *red = reinterpret_cast<double *>(b + red_off);
  double *d_norm = red + reduction_partials_needed();
  hipStream_t st = reinterpret_cast<hipStream_t>(s);
  if (x0) {
    CT_TRY_HIP(hipMemcpyAsync(x, x0, img_bytes, hipMemcpyDeviceToDevice, st));
  } else {
    hipLaunchKernelGGL(k_default_start, dim3((n + 255) / 256, n), dim3(256), 0, st, n, x);
    CT_TRY_HIP(hipGetLastError());
  }
  // x <- x / ||x||; per step x <- R^*(R x) / ||R^*(R x)||, the estimate being
  // the last norm (R^* with one angle slice: it writes x directly, after R
  // has read it)
  CT_TRY(launch_norm2(x, (int64_t)nn, red, red_cap, d_norm, st));
  CT_TRY(launch_scale_by_inv(x, (int64_t)nn, d_norm, x, st));
  for (int it = 0; it < iters; ++it) {
    CT_TRY(launch_radon_fwd(p, x, sino, st));
    CT_TRY(launch_radon_adj(p, sino, nullptr, 1.0f, 0.0f, x, st, 1, nullptr, 1));
    CT_TRY(launch_norm2(x, (int64_t)nn, red, red_cap, d_norm, st));
    CT_TRY(launch_scale_by_inv(x, (int64_t)nn, d_norm, x, st));
  }
  double lam = 0.0;
  CT_TRY_HIP(hipMemcpyAsync(&lam, d_norm, sizeof(double), hipMemcpyDeviceToHost, st));
  CT_TRY_HIP(hipStreamSynchronize(st));
  *out = std::sqrt(lam);
  return CT_OK;
}
