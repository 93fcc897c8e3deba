// Measurement utilities, not steps of the method: a probe of the vector
// (VALU) issue rate and a streaming device copy, with which the nominal
// rates behind the projectors' and the preconditioner's rooflines are
// checked on the device at hand.
#include "common.hpp"

namespace ctpd {

constexpr int kProbeThreads = 256;
constexpr int kProbeChains = 16;  // independent FMA chains per lane

// Each lane runs kProbeChains independent chains for `iters` rounds (the
// round loop is scalar), so the launch issues blocks * 4 * iters *
// kProbeChains * I wave-instructions of the kind KIND, I per chain and round:
// 0 FP32 FMA (v_fma_f32, I = 1), 1 FP32 add (v_add_f32, I = 1), 2 32-bit
// integer xor-add (v_xad_u32, I = 1), 3 xor-add and integer-to-float
// conversion feeding each other (v_xad_u32 + v_cvt_f32_u32, I = 2), 4 64-bit
// integer add (v_lshl_add_u64, I = 1; the step is made opaque to the compiler
// each round so that the sum stays a chain of adds).  The chains stay finite
// and non-negative; the conditional store only keeps them live.
template <int KIND>
__global__ __launch_bounds__(kProbeThreads) void k_valu_probe(int iters, float seed,
                                                              float *__restrict__ out) {
  const float m = 1.0f - 1.0e-7f * (float)(threadIdx.x & 7);
  const uint32_t step = 1u + (threadIdx.x & 7), key = 0x9e3779b9u * (threadIdx.x + 1u);
  float a[kProbeChains];
  uint32_t b[kProbeChains];
  uint64_t d[kProbeChains];
  uint64_t step64 = step;
#pragma unroll
  for (int c = 0; c < kProbeChains; ++c) {
    a[c] = seed * (float)(c + 1);
    b[c] = (uint32_t)c * 977u + threadIdx.x;
    d[c] = b[c];
  }
  for (int it = 0; it < iters; ++it) {
    if constexpr (KIND == 4) asm volatile("" : "+v"(step64));
#pragma unroll
    for (int c = 0; c < kProbeChains; ++c) {
      if constexpr (KIND == 0) {
        a[c] = fmaf(a[c], m, seed);
      } else if constexpr (KIND == 1) {
        a[c] = a[c] + m;
      } else if constexpr (KIND == 2) {
        b[c] = (b[c] ^ key) + step;
      } else if constexpr (KIND == 3) {
        b[c] = (b[c] ^ __float_as_uint(a[c])) + step;
        a[c] = (float)b[c];
      } else {
        d[c] = d[c] + step64;
      }
    }
  }
  float s = 0.f;
#pragma unroll
  for (int c = 0; c < kProbeChains; ++c)
    s += KIND == 2 ? (float)b[c] : KIND == 4 ? (float)(uint32_t)(d[c] >> 8) : a[c];
  // every chain stays >= 0 and the launcher passes seed > 0, so this is
  // never taken; the compiler cannot know seed's sign and keeps the chains
  if (s == -seed) out[blockIdx.x] = s;
}

// dst[i] = src[i] for n16 16-byte elements, grid-strided.
__global__ __launch_bounds__(kProbeThreads) void k_copy16(const float4 *__restrict__ src,
                                                          float4 *__restrict__ dst, long long n16) {
  const long long stride = (long long)gridDim.x * kProbeThreads;
  for (long long i = (long long)blockIdx.x * kProbeThreads + threadIdx.x; i < n16; i += stride)
    dst[i] = src[i];
}

}  // namespace ctpd

extern "C" int ct_valu_probe(int32_t blocks, int32_t iters, int32_t kind, float *out,
                             ct_stream s) {
  using namespace ctpd;
  if (blocks < 1 || iters < 1 || kind < 0 || kind > 4 || out == nullptr) {
    set_error("ct_valu_probe: need blocks >= 1, iters >= 1, kind 0..4 and an output buffer");
    return CT_E_INVALID;
  }
  const dim3 grid(blocks), block(kProbeThreads);
  const hipStream_t st = (hipStream_t)s;
  if (kind == 0)
    hipLaunchKernelGGL(k_valu_probe<0>, grid, block, 0, st, iters, 1.0e-3f, out);
  else if (kind == 1)
    hipLaunchKernelGGL(k_valu_probe<1>, grid, block, 0, st, iters, 1.0e-3f, out);
  else if (kind == 2)
    hipLaunchKernelGGL(k_valu_probe<2>, grid, block, 0, st, iters, 1.0e-3f, out);
  else if (kind == 3)
    hipLaunchKernelGGL(k_valu_probe<3>, grid, block, 0, st, iters, 1.0e-3f, out);
  else
    hipLaunchKernelGGL(k_valu_probe<4>, grid, block, 0, st, iters, 1.0e-3f, out);
  CT_TRY_HIP(hipGetLastError());
  return CT_OK;
}

extern "C" int ct_copy_probe(const void *src, void *dst, int64_t bytes, int32_t blocks,
                             ct_stream s) {
  using namespace ctpd;
  if (src == nullptr || dst == nullptr || bytes < 16 || bytes % 16 != 0 || blocks < 1 ||
      (reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) % 16 != 0) {
    set_error("ct_copy_probe: need 16-byte aligned buffers, a size that is a positive "
              "multiple of 16 and blocks >= 1");
    return CT_E_INVALID;
  }
  hipLaunchKernelGGL(k_copy16, dim3(blocks), dim3(kProbeThreads), 0, (hipStream_t)s,
                     static_cast<const float4 *>(src), static_cast<float4 *>(dst),
                     (long long)(bytes / 16));
  CT_TRY_HIP(hipGetLastError());
  return CT_OK;
}
