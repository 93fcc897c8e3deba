// Discrete Radon pair R_h / R_h^* on gfx950 (thesis §3.1).
//
// Both kernels evaluate the bin coordinate of pixel (i, j) at angle l,
//   t = (x_i cos theta_l + y_j sin theta_l)/ds + (M-1)/2,
// from constants quantized to multiples of 2^-30, so t itself is an exact
// multiple of 2^-30: the backprojection evaluates it exactly in FP64, the
// forward projection exactly in integers.  The interpolation weight
// alpha = t - floor(t) is rounded once to FP32 in both, giving bit-identical
// weights; R_h is the transpose of R_h^* up to FP32 summation order.
#include <type_traits>

#include "common.hpp"
#include "tv_update.hpp"

namespace ctpd {

// clamp x to [lo, hi] in one instruction
__device__ inline int med3i(int x, int lo, int hi) {
  int r;
  asm("v_med3_i32 %0, %1, %2, %3" : "=v"(r) : "v"(x), "v"(lo), "v"(hi));
  return r;
}

// Word 3 of a raw buffer descriptor (32-bit data).  Buffer loads are range
// checked: a load whose byte offset is not below the descriptor's record
// count returns 0, a documented property of buffer addressing; both kernels
// stage through such loads to get the zeros off the image or detector.
constexpr int kBufWord3 = 0x00020000;

// A buffer-load byte offset kept in a register of its own: the range check
// must see exactly this value, so no constant part of it may be moved into
// the instruction's immediate offset field.
__device__ inline int own_offset(int off) {
  asm volatile("" : "+v"(off));
  return off;
}

// ---------------------------------------------------------------------------
// R_h^*: pixel-driven gather.
//
// One workgroup per kBpTileI x kBpTileJ pixel tile and per angle slice (the
// angles are split over gridDim.z slices whose partial images are summed,
// with the epilogue, by the preconditioner's FFT row pass or by k_bp_combine
// when there is more than one).  Thread (tx, ty) owns the
// kBpPix pixels (i0 + tx, j0 + ty + 8 p).  For every chunk of kBpChunk angles
// the detector segment the tile projects onto is staged in LDS as pairs
// (v[k], v[k+1] - v[k]).  Per angle a thread evaluates its first pixel's
// bin coordinate exactly in FP64, splits it into a local bin index (hi) and a
// 32-bit fraction (lo), then steps to its other pixels with exact 64-bit
// integer additions of 8 b 2^32.  alpha = lo 2^-32 is rounded once to FP32,
// the same rounding as the forward projector's.
//
// The first pixel's coordinate is formed as the double 2^52 + t 2^32, where
// t is relative to the staged segment: it is an integer in [2^52, 2^53)
// (t is a multiple of 2^-30 in [0, seg)), so the FMAs that form it are exact
// and its bit pattern is the 64-bit fixed-point value itself, offset by the
// exponent field in the high word (kMagicHi, folded into the LDS base).
constexpr uint32_t kMagicHi = 0x43300000u;  // high word of the double 2^52

// Constants of one coordinate chain in LDS (read by the angle loops with
// in-order LDS loads rather than scalar loads): 2^52 + (t0 - kmin) 2^32,
// a 2^32, b 2^32 and the per-pixel step 8 b 2^32.
struct alignas(16) ChainGeo {
  double tb, a32, b32;
  int64_t b8;
};

__device__ inline void bp_chunk_meta(const BpAngle *__restrict__ ang, int c0, int nc, int i0, int j0,
                                     int *kmin_s, int *row_s, ChainGeo *geo_s) {
  if ((int)threadIdx.x < nc) {
    const BpAngle A = ang[c0 + threadIdx.x];
    const double ic = (A.a >= 0.0) ? (double)i0 : (double)(i0 + kBpTileI - 1);
    const double jc = (A.b >= 0.0) ? (double)j0 : (double)(j0 + kBpTileJ - 1);
    const double tmin = fma(jc, A.b, fma(ic, A.a, A.t0));
    const int kmin = (int)floor(tmin);
    kmin_s[threadIdx.x] = kmin;
    row_s[threadIdx.x] = A.l;
    // 2^52 + (t0 - kmin) 2^32: every term and partial sum is an integer below 2^53
    geo_s[threadIdx.x] = ChainGeo{fma(A.t0 - (double)kmin, 4294967296.0, 4503599627370496.0),
                                  A.a32, A.b32, A.b8_fix};
  }
}

// Segment values of one chunk into registers.  Wave w stages the angles
// c = w + 4 r of the chunk, each through a buffer descriptor covering just
// that angle's sinogram row, so bins off the detector (a negative bin wraps
// to a huge byte offset) and angles past the chunk's end (record count 0)
// read as 0 without branches or masks.  Lane t holds the pairs
// (v[k], v[k+1]) for the local bins k = t and k = t + 64 of each angle.
constexpr int kBpWaves = 4;                                  // 256 threads
constexpr int kBpAnglesPerWave = kBpChunk / kBpWaves;        // 4
constexpr int kBpBinRounds = kBpPrefetch / kBpAnglesPerWave; // 2: seg <= 128
static_assert(kBpAnglesPerWave * kBpBinRounds == kBpPrefetch, "staging layout");
static_assert(64 * kBpBinRounds * kBpChunk == 256 * kBpPrefetch, "staging covers seg <= 128");

__device__ inline void bp_stage_load(float2 (&v)[kBpPrefetch], const float *__restrict__ sino,
                                     int M, int nc, const int *kmin_s, const int *row_s) {
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int r = 0; r < kBpAnglesPerWave; ++r) {
    const int c = w + kBpWaves * r;  // wave-uniform
    const int cc = min(c, nc - 1);
    const int row = __builtin_amdgcn_readfirstlane(row_s[cc]);
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        (void *)(sino + (size_t)row * M), (short)0, c < nc ? M * 4 : 0, kBufWord3);
    const int k0 = kmin_s[cc] + lane;
#pragma unroll
    for (int m = 0; m < kBpBinRounds; ++m) {
      const int k = k0 + 64 * m;
      // every load keeps its own offset register (a negative bin is a huge
      // unsigned offset, out of range): no folding of the +4 or +256 into a
      // merged or immediate-offset load, whose range check would differ at
      // the detector's ends
      const float v0 =
          __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, own_offset(k * 4), 0, 0));
      const float v1 =
          __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, own_offset(k * 4 + 4), 0, 0));
      v[r * kBpBinRounds + m] = make_float2(v0, v1);
    }
  }
}

// LDS entry c seg + k holds (v[k], v[k+1] - v[k]) of angle c, bin kmin_c + k.
__device__ inline void bp_stage_store(const float2 (&v)[kBpPrefetch], float2 *vd, int seg,
                                      int nc) {
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
  for (int r = 0; r < kBpAnglesPerWave; ++r) {
    const int c = w + kBpWaves * r;
#pragma unroll
    for (int m = 0; m < kBpBinRounds; ++m) {
      const int k = lane + 64 * m;
      const float2 q = v[r * kBpBinRounds + m];
      if (c < nc && k < seg) vd[c * seg + k] = make_float2(q.x, q.y - q.x);
    }
  }
}

// gridDim.z = (problems of a batch) x S angle slices: problem b = z / S.
__global__ __launch_bounds__(256) void k_radon_adj(
    const float *__restrict__ sino, int n, int N, int M, const BpAngle *__restrict__ ang,
    int seg, int slice_len, int S, const float *__restrict__ pfield, float c1, float c2,
    float inv_h, const float *__restrict__ base, const float *__restrict__ base2,
    float *__restrict__ out, float *__restrict__ out2) {
  extern __shared__ float2 vd_all[];  // 2 x kBpChunk * seg
  __shared__ int row_s[3][kBpChunk];
  __shared__ int kmin_s[3][kBpChunk];
  __shared__ ChainGeo geo_s[3][kBpChunk];
  const int tx = threadIdx.x & (kBpTileI - 1);
  const int ty = threadIdx.x / kBpTileI;  // 0..7
  const int i0 = blockIdx.x * kBpTileI, j0 = blockIdx.y * kBpTileJ;
  const int i = i0 + tx;
  const int jb = j0 + ty;
  double di = (double)i, dj = (double)jb;
  asm volatile("" : "+v"(di), "+v"(dj));  // converted once, not per angle
  const int bz = blockIdx.z / S, sl = blockIdx.z - bz * S;
  const size_t nn = (size_t)n * n;
  sino += (size_t)bz * N * M;
  if (pfield != nullptr) pfield += (size_t)bz * 2 * nn;
  if (base != nullptr) base += (size_t)bz * nn;
  if (base2 != nullptr) base2 += (size_t)bz * nn;
  if (out2 != nullptr) out2 += (size_t)bz * nn;
  out += (size_t)blockIdx.z * nn;  // own image (S == 1) or own partial image
  const int a_begin = sl * slice_len;
  const int a_end = min(N, a_begin + slice_len);
  const int nchunks = a_end > a_begin ? (a_end - a_begin + kBpChunk - 1) / kBpChunk : 0;
  float accv[kBpPix], accd[kBpPix];
#pragma unroll
  for (int p = 0; p < kBpPix; ++p) {
    accv[p] = 0.f;
    accd[p] = 0.f;
  }

  // Chunk it's detector segments are double-buffered in LDS (the chunk
  // metadata triple-buffered); chunk it+1 is loaded into registers while
  // chunk it is interpolated.
  float2 pf[kBpPrefetch];
  if (nchunks > 0) {
    bp_chunk_meta(ang, a_begin, min(kBpChunk, a_end - a_begin), i0, j0, kmin_s[0], row_s[0],
                  geo_s[0]);
    __syncthreads();
    bp_stage_load(pf, sino, M, min(kBpChunk, a_end - a_begin), kmin_s[0], row_s[0]);
  }
  for (int it = 0; it < nchunks; ++it) {
    const int c0 = a_begin + it * kBpChunk;
    const int nc = min(kBpChunk, a_end - c0);
    const int slot = it % 3;
    float2 *vd = vd_all + (it & 1) * (kBpChunk * seg);
    bp_stage_store(pf, vd, seg, nc);
    const int c1n = c0 + kBpChunk;
    const int ncn = min(kBpChunk, a_end - c1n);
    if (it + 1 < nchunks)
      bp_chunk_meta(ang, c1n, ncn, i0, j0, kmin_s[(it + 1) % 3], row_s[(it + 1) % 3],
                    geo_s[(it + 1) % 3]);
    __syncthreads();
    if (it + 1 < nchunks)
      bp_stage_load(pf, sino, M, ncn, kmin_s[(it + 1) % 3], row_s[(it + 1) % 3]);
    for (int c = 0; c < nc; ++c) {
      const ChainGeo G = geo_s[slot][c];
      // first pixel: 2^52 + t 2^32 with t relative to the staged segment (exact)
      const double x = fma(dj, G.b32, fma(di, G.a32, G.tb));
      uint64_t tf = (uint64_t)__double_as_longlong(x);
      const uint64_t step = (uint64_t)G.b8;  // 8 b 2^32, exact
      const float2 *seg_c = vd + c * seg;
      // the high word is kMagicHi + the local bin index, in [0, seg - 2] by construction
      uint32_t hh[kBpPix];
      uint32_t ll[kBpPix];
#pragma unroll
      for (int p = 0; p < kBpPix; ++p) {
        if (p > 0) {
          tf += step;                    // one 64-bit add per pixel
          asm volatile("" : "+v"(tf));   // keep the chain (no rewrite into multiplies)
        }
        hh[p] = (uint32_t)(tf >> 32);
        ll[p] = (uint32_t)tf;
      }
      float2 q[kBpPix];
#pragma unroll
      for (int p = 0; p < kBpPix; ++p) q[p] = seg_c[(int)(hh[p] - kMagicHi)];
#pragma unroll
      for (int p = 0; p < kBpPix; ++p) {
        accv[p] += q[p].x;
        accd[p] = fmaf((float)ll[p], q[p].y, accd[p]);
      }
    }
  }
  const float inv32 = 2.3283064365386963e-10f;  // 2^-32
  const bool final_out = (S == 1);
#pragma unroll
  for (int p = 0; p < kBpPix; ++p) {
    const int j = jb + kBpRowStep * p;
    if (i >= n || j >= n) continue;
    const size_t o = (size_t)j * n + i;
    const float r = fmaf(accd[p], inv32, accv[p]);
    if (!final_out) {
      out[o] = r;
      continue;
    }
    float res = c1 * r;
    if (pfield != nullptr) {
      const float *p1 = pfield;
      const float *p2 = pfield + (size_t)n * n;
      const float d1 = (i < n - 1 ? p1[o] : 0.f) - (i > 0 ? p1[o - 1] : 0.f);
      const float d2 = (j < n - 1 ? p2[o] : 0.f) - (j > 0 ? p2[o - n] : 0.f);
      res = fmaf(c2 * inv_h, d1 + d2, res);
    }
    if (base != nullptr) res += base[o];
    if (base2 != nullptr) res -= base2[o];
    out[o] = res;
    if (out2 != nullptr) out2[o] = 2.f * res - base[o];
  }
}

// out = base - base2 + c1 * sum_s part[s] + c2 * div_h(p): the angle slices' partial
// backprojections summed in slice order, with the same epilogue.
__global__ void k_bp_combine(const float *__restrict__ part, int S, int n,
                             const float *__restrict__ pfield, float c1, float c2, float inv_h,
                             const float *__restrict__ base, const float *__restrict__ base2,
                             float *__restrict__ out, float *__restrict__ out2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (i >= n) return;
  const size_t o = (size_t)j * n + i, nn = (size_t)n * n;
  part += (size_t)blockIdx.z * S * nn;  // problem blockIdx.z of a batch
  if (pfield != nullptr) pfield += (size_t)blockIdx.z * 2 * nn;
  if (base != nullptr) base += (size_t)blockIdx.z * nn;
  if (base2 != nullptr) base2 += (size_t)blockIdx.z * nn;
  if (out2 != nullptr) out2 += (size_t)blockIdx.z * nn;
  out += (size_t)blockIdx.z * nn;
  float r = part[o];
  for (int s = 1; s < S; ++s) r += part[s * nn + o];
  float res = c1 * r;
  if (pfield != nullptr) {
    const float *p1 = pfield;
    const float *p2 = pfield + nn;
    const float d1 = (i < n - 1 ? p1[o] : 0.f) - (i > 0 ? p1[o - 1] : 0.f);
    const float d2 = (j < n - 1 ? p2[o] : 0.f) - (j > 0 ? p2[o - n] : 0.f);
    res = fmaf(c2 * inv_h, d1 + d2, res);
  }
  if (base != nullptr) res += base[o];
  if (base2 != nullptr) res -= base2[o];
  out[o] = res;
  if (out2 != nullptr) out2[o] = 2.f * res - base[o];
}

// ---------------------------------------------------------------------------
// R_h^* over mirror pairs (theta_l, theta_m = pi - theta_l).
//
// Angle m puts pixel (n - 1 - i, j) exactly where l puts pixel (i, j), so one
// bin coordinate serves two (pixel, angle) terms.  A workgroup owns a tile of
// the left half (i < ceil(n/2)) and its mirror image; a thread evaluates two
// coordinate chains per pair over its pixels (i, j_p):
//   chain 0: t(i, j; l)  = t(n-1-i, j; m)  -> v_l to pixel L, v_m to pixel R
//   chain 1: t(i, j; m)  = t(n-1-i, j; l)  -> v_m to pixel L, v_l to pixel R
// Each chain has its own staged detector segment, holding for every bin both
// angles' (v[k], v[k+1] - v[k]), at a constant distance from each other (two
// single 8-byte LDS reads from one address; paired ds_read2 forms measured
// slower).  An angle without a partner runs with its mirror image's geometry
// and a zero sinogram row.  On the centre column of an odd n (i = n - 1 - i)
// the L terms already hold both angles, and the R terms are dropped.  Tiles
// are kBpTileI x 8 PIX: with PIX = 4, more workgroups than the one-angle
// kernel's tiles at a register count that keeps them resident; with PIX = 8
// the one-angle kernel's tiles (less staging per pixel, for large grids).

// Staging of the mirror-pair kernel.  R rounds of 64 bins cover a segment
// (R = 1: seg <= 64, R = 2: seg <= 128); a chunk holds kBpPrefetch / R pairs,
// so that every thread stages kBpPrefetch (v[k], v[k+1]) pairs per chunk.
// LDS float2 entry a kSlot + (2c + g) 64 R + k holds (v[k], v[k+1] - v[k]) of
// angle slot a (0: l, 1: m) of pair c on chain g's segment: the two angles of
// a bin are read with one address and a constant offset.
template <int R, int PIX>
struct PairStage {
  static constexpr int kTileJ = kBpRowStep * PIX;  // tile rows (PIX pixels per thread)
  static constexpr int kPairs = kBpPrefetch / R;  // pairs per chunk
  static constexpr int kStride = 64 * R;          // entries per (pair, chain, slot)
  // slot 1's offset: neither within a ds_read2_b64's reach nor a multiple of
  // 64 entries, so the two angles' reads stay single ds_read_b64 instructions
  static constexpr int kSlot = kPairs * 2 * kStride + 8;

  // Per pair c and chain g: segment start, the sinogram row of slot g (entry
  // 2c + g of the pair table) and, for the coordinate chain, 2^52 + (t0 -
  // kmin) 2^32, a 2^32, b 2^32 and 8 b 2^32 -- in LDS, so that the pair loop
  // reads them with in-order LDS loads instead of scalar loads.
  __device__ static void meta(const BpAngle *__restrict__ pang, int c0, int nc, int i0, int j0,
                              int *kmin_s, int *row_s, ChainGeo *geo_s) {
    const int t = threadIdx.x;
    if (t < 2 * nc) {
      const BpAngle A = pang[2 * c0 + t];
      const double ic = (A.a >= 0.0) ? (double)i0 : (double)(i0 + kBpTileI - 1);
      const double jc = (A.b >= 0.0) ? (double)j0 : (double)(j0 + kTileJ - 1);
      const double tmin = fma(jc, A.b, fma(ic, A.a, A.t0));
      const int kmin = (int)floor(tmin);
      kmin_s[t] = kmin;
      row_s[t] = A.l;
      geo_s[t] = ChainGeo{fma(A.t0 - (double)kmin, 4294967296.0, 4503599627370496.0), A.a32,
                          A.b32, A.b8_fix};
    }
  }

  // Wave w stages chain g = w >> 1 of slot a = w & 1 for every pair of the
  // chunk, through a descriptor covering the slot's sinogram row (record
  // count 0 for a missing partner or a pair past the chunk's end).
  __device__ static void load(float2 (&v)[kBpPrefetch], const float *__restrict__ sino, int M,
                              int nc, const int *kmin_s, const int *row_s) {
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int g = w >> 1, a = w & 1;
#pragma unroll
    for (int c = 0; c < kPairs; ++c) {
      const int cc = min(c, nc - 1);
      const int row = __builtin_amdgcn_readfirstlane(row_s[2 * cc + a]);
      const bool ok = c < nc && row >= 0;
      const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
          (void *)(sino + (size_t)(ok ? row : 0) * M), (short)0, ok ? M * 4 : 0, kBufWord3);
      const int k0 = kmin_s[2 * cc + g] + lane;
#pragma unroll
      for (int m = 0; m < R; ++m) {
        const int k = k0 + 64 * m;
        const float v0 =
            __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, own_offset(k * 4), 0, 0));
        const float v1 =
            __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, own_offset(k * 4 + 4), 0, 0));
        v[c * R + m] = make_float2(v0, v1);
      }
    }
  }

  __device__ static void store(const float2 (&v)[kBpPrefetch], float2 *vd, int seg, int nc) {
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int g = w >> 1, a = w & 1;
#pragma unroll
    for (int c = 0; c < kPairs; ++c) {
#pragma unroll
      for (int m = 0; m < R; ++m) {
        const int k = lane + 64 * m;
        const float2 q = v[c * R + m];
        if (c < nc && k < seg) vd[a * kSlot + (2 * c + g) * kStride + k] = make_float2(q.x, q.y - q.x);
      }
    }
  }
};

// Tile of workgroup (bx, by) of the gx x gy tiles of a z-slice.  Workgroups
// are dealt to the 8 XCDs in turn by linear index; where gy is a multiple of
// 8, the workgroups that land on XCD x take the tile rows of the x-th eighth
// of the image (a bijection of the grid onto itself): the tiles of one band
// read overlapping detector segments of every angle and so share their XCD's
// L2.
__device__ inline void xcd_row_tile(int &bx, int &by) {
  const int gx = gridDim.x, gy = gridDim.y;
  if ((gy & 7) != 0) return;
  const int L = bx + gx * by;
  const int x = L & 7, k = L >> 3;
  const int q = k / gx;
  by = x * (gy >> 3) + q;
  bx = k - q * gx;
}

// gridDim.z = (problems of a batch) x S slices of the pairs: problem b = z / S.
// PIX pixels per thread: tiles of kBpTileI x 8 PIX.
template <int R, int PIX>
__global__ __launch_bounds__(256) void k_radon_adj_pair(
    const float *__restrict__ sino, int n, int N, int M, const BpAngle *__restrict__ pang,
    int seg, int slice_len, int S, const float *__restrict__ pfield, float c1, float c2,
    float inv_h, const float *__restrict__ base, const float *__restrict__ base2,
    float *__restrict__ out, float *__restrict__ out2, int n_pairs) {
  using PS = PairStage<R, PIX>;
  constexpr int kPairs = PS::kPairs, kStride = PS::kStride, kSlot = PS::kSlot;
  __shared__ float2 vq_all[2 * 2 * kSlot];  // 2 buffers x 2 slots x pairs x 2 chains
  __shared__ int row_s[3][2 * kPairs];
  __shared__ int kmin_s[3][2 * kPairs];
  __shared__ ChainGeo geo_s[3][2 * kPairs];
  const int tx = threadIdx.x & (kBpTileI - 1);
  const int ty = threadIdx.x / kBpTileI;  // 0..7
  int bx = blockIdx.x, by = blockIdx.y;
  xcd_row_tile(bx, by);
  const int i0 = bx * kBpTileI, j0 = by * PS::kTileJ;
  const int i = i0 + tx;  // left-half column; its mirror is n - 1 - i
  const int jb = j0 + ty;
  double di = (double)i, dj = (double)jb;
  asm volatile("" : "+v"(di), "+v"(dj));  // converted once, not per pair
  const int bz = blockIdx.z / S, sl = blockIdx.z - bz * S;
  const size_t nn = (size_t)n * n;
  sino += (size_t)bz * N * M;
  if (pfield != nullptr) pfield += (size_t)bz * 2 * nn;
  if (base != nullptr) base += (size_t)bz * nn;
  if (base2 != nullptr) base2 += (size_t)bz * nn;
  if (out2 != nullptr) out2 += (size_t)bz * nn;
  out += (size_t)blockIdx.z * nn;  // own image (S == 1) or own partial image
  const int c_begin = sl * slice_len;
  const int c_end = min(n_pairs, c_begin + slice_len);
  const int nchunks =
      c_end > c_begin ? (c_end - c_begin + kPairs - 1) / kPairs : 0;
  float lv[PIX], ld[PIX], rv[PIX], rd[PIX];
#pragma unroll
  for (int p = 0; p < PIX; ++p) lv[p] = ld[p] = rv[p] = rd[p] = 0.f;

  float2 pf[kBpPrefetch];
  if (nchunks > 0) {
    PS::meta(pang, c_begin, min(kPairs, c_end - c_begin), i0, j0, kmin_s[0], row_s[0],
             geo_s[0]);
    __syncthreads();
    PS::load(pf, sino, M, min(kPairs, c_end - c_begin), kmin_s[0], row_s[0]);
  }
  for (int it = 0; it < nchunks; ++it) {
    const int c0 = c_begin + it * kPairs;
    const int nc = min(kPairs, c_end - c0);
    const int slot = it % 3;
    float2 *vq = vq_all + (it & 1) * (2 * kSlot);
    PS::store(pf, vq, seg, nc);
    const int c1n = c0 + kPairs;
    const int ncn = min(kPairs, c_end - c1n);
    if (it + 1 < nchunks)
      PS::meta(pang, c1n, ncn, i0, j0, kmin_s[(it + 1) % 3], row_s[(it + 1) % 3],
               geo_s[(it + 1) % 3]);
    __syncthreads();
    if (it + 1 < nchunks)
      PS::load(pf, sino, M, ncn, kmin_s[(it + 1) % 3], row_s[(it + 1) % 3]);
#pragma unroll 2
    for (int c = 0; c < nc; ++c) {
      const ChainGeo G0 = geo_s[slot][2 * c], G1 = geo_s[slot][2 * c + 1];
      const double x0 = fma(dj, G0.b32, fma(di, G0.a32, G0.tb));
      const double x1 = fma(dj, G1.b32, fma(di, G1.a32, G1.tb));
      const uint64_t step = (uint64_t)G0.b8;  // b is the same for both chains
      // one chain at a time: v_l and v_m go to (L, R) on chain 0, (R, L) on chain 1
      auto chain = [&](double x, const float2 *sg, float *va, float *da, float *vb, float *db) {
        // the high word less the exponent field: the local bin index itself
        uint64_t f = (uint64_t)__double_as_longlong(x) - ((uint64_t)kMagicHi << 32);
        uint32_t hh[PIX], ll[PIX];
#pragma unroll
        for (int p = 0; p < PIX; ++p) {
          if (p > 0) {
            f += step;
            asm("" : "+v"(f));
          }
          hh[p] = (uint32_t)(f >> 32);
          ll[p] = (uint32_t)f;
        }
        float2 qa[PIX], qb[PIX];
#pragma unroll
        for (int p = 0; p < PIX; ++p) {
          qa[p] = sg[hh[p]];          // angle l
          qb[p] = sg[hh[p] + kSlot];  // angle m
        }
#pragma unroll
        for (int p = 0; p < PIX; ++p) {
          const float al = (float)ll[p];
          va[p] += qa[p].x;
          da[p] = fmaf(al, qa[p].y, da[p]);
          vb[p] += qb[p].x;
          db[p] = fmaf(al, qb[p].y, db[p]);
        }
      };
      chain(x0, vq + (2 * c) * kStride, lv, ld, rv, rd);
      chain(x1, vq + (2 * c + 1) * kStride, rv, rd, lv, ld);
    }
  }
  const float inv32 = 2.3283064365386963e-10f;  // 2^-32
  const bool final_out = (S == 1);
  const int nh = (n + 1) / 2;
  if (i >= nh) return;
  const int ir = n - 1 - i;
  auto emit = [&](int col, int j, float r) {
    const size_t o = (size_t)j * n + col;
    if (!final_out) {
      out[o] = r;
      return;
    }
    float res = c1 * r;
    if (pfield != nullptr) {
      const float *p1 = pfield;
      const float *p2 = pfield + nn;
      const float d1 = (col < n - 1 ? p1[o] : 0.f) - (col > 0 ? p1[o - 1] : 0.f);
      const float d2 = (j < n - 1 ? p2[o] : 0.f) - (j > 0 ? p2[o - n] : 0.f);
      res = fmaf(c2 * inv_h, d1 + d2, res);
    }
    if (base != nullptr) res += base[o];
    if (base2 != nullptr) res -= base2[o];
    out[o] = res;
    if (out2 != nullptr) out2[o] = 2.f * res - base[o];
  };
#pragma unroll
  for (int p = 0; p < PIX; ++p) {
    const int j = jb + kBpRowStep * p;
    if (j >= n) continue;
    emit(i, j, fmaf(ld[p], inv32, lv[p]));
    if (ir != i) emit(ir, j, fmaf(rd[p], inv32, rv[p]));
  }
}

int launch_radon_adj(const ct_plan *p, const float *v, const float *pfield, float c1,
                     float c2, float *out, hipStream_t s, int nb, float *part, int S, int kern,
                     const float *base, const float *base2, float *out2, BpDeferred *defer) {
  const int n = p->g.n;
  if (S <= 0) S = p->bp_slices;
  if (defer) *defer = BpDeferred{};
  const int slice_len = (p->g.n_angles + S - 1) / S;
  if (nb < 1 || (S > 1 && part == nullptr && (nb > 1 || S > p->bp_slices))) {
    set_error("backprojection: batch needs its own partial-image buffer");
    return CT_E_INVALID;
  }
  if (part == nullptr) part = p->d_bp_part;
  float *dst = (S == 1) ? out : part;
  if (kern < 0) kern = p->bp_kern0;
  if (p->n_bpp > 0 && kern != 0) {
    const int nh = (n + 1) / 2;
    const int pair_len = (p->n_bpp + S - 1) / S;
    // 4 pixels per thread on 32 x 32 tiles, or 8 on 32 x 64 (the one-angle
    // kernel's tile, whose segment length it shares)
    const int pix = kern == 8 ? 8 : 4;
    const int seg = pix == 8 ? p->seg : p->seg_pair;
    dim3 grid((nh + kBpTileI - 1) / kBpTileI, (n + kBpRowStep * pix - 1) / (kBpRowStep * pix),
              S * nb);
    auto go = [&](auto r_c, auto pix_c) {
      constexpr int RR = decltype(r_c)::value, PP = decltype(pix_c)::value;
      hipLaunchKernelGGL((k_radon_adj_pair<RR, PP>), grid, dim3(256), 0, s, v, n, p->g.n_angles,
                         p->g.n_bins, p->d_bpp, seg, pair_len, S, pfield, c1, c2,
                         (float)(1.0 / p->g.h), base, base2, dst, S == 1 ? out2 : nullptr,
                         p->n_bpp);
    };
    using I1 = std::integral_constant<int, 1>;
    using I2 = std::integral_constant<int, 2>;
    using P4 = std::integral_constant<int, 4>;
    using P8 = std::integral_constant<int, 8>;
    if (pix == 4) {
      if (seg <= 64) go(I1{}, P4{});
      else go(I2{}, P4{});
    } else {
      if (seg <= 64) go(I1{}, P8{});
      else go(I2{}, P8{});
    }
  } else {
    dim3 grid((n + kBpTileI - 1) / kBpTileI, (n + kBpTileJ - 1) / kBpTileJ, S * nb);
    const size_t lds = 2 * sizeof(float2) * kBpChunk * p->seg;
    hipLaunchKernelGGL(k_radon_adj, grid, dim3(256), lds, s, v, n, p->g.n_angles, p->g.n_bins,
                       p->d_bp, p->seg, slice_len, S, pfield, c1, c2, (float)(1.0 / p->g.h),
                       base, base2, dst, S == 1 ? out2 : nullptr);
  }
  CT_TRY_HIP(hipGetLastError());
  if (defer != nullptr && out2 == nullptr && deferrable_slices(S)) {
    // the consumer forms out from the partial images
    *defer = BpDeferred{part, S, pfield, c1, c2, (float)(1.0 / p->g.h), base, base2};
    return CT_OK;
  }
  if (S > 1) {
    hipLaunchKernelGGL(k_bp_combine, dim3((n + 255) / 256, n, nb), dim3(256), 0, s, part, S, n,
                       pfield, c1, c2, (float)(1.0 / p->g.h), base, base2, out, out2);
    CT_TRY_HIP(hipGetLastError());
  }
  return CT_OK;
}

// ---------------------------------------------------------------------------
// R_h: ray-driven gather with an exact integer walk.
//
// In the walk frame (image transposed and/or mirrored per angle class) the
// fixed-point coordinate is t(p, q) = T + p A + q B with A > 0, 0 <= B <= A.
// Strip k of a row q is the set of pixels with floor(t) = k: it starts at
// p_s = ceil((k 2^30 - T - q B)/A) and holds one or two pixels (A >= 2^29).
// Its pixels give weight 1 - alpha to bin k and alpha to bin k+1, so with
//   P_k = sum_strip u,   Q_k = sum_strip alpha u,
// bin k receives R[k] = P_k - Q_k + Q_{k-1}.  Each lane owns strip k and walks
// all rows: e = t(p_s, q) - k 2^30 is kept exactly in [0, A); one row down,
// e += B, and if e >= A the strip starts one pixel earlier (e -= A).
// A workgroup owns kFpGroup angles of one class (kFpPerThread per wave) and
// kFpStrips consecutive strips; image rows are staged in LDS kFpRows at a
// time over the column range precomputed on the host for that
// (group, block, chunk).  Lane 0's strip only supplies Q_{k-1} to lane 1.

// Problem blockIdx.z of a batch: images [n][n], sinograms [N][M] and masks
// [N][ceil(M/32)] follow each other contiguously.
__device__ inline void fp_batch_offsets(const float *__restrict__ &u, float *__restrict__ &sino,
                                        SinoEpi &ep, int n, int N, int M) {
  const size_t b = blockIdx.z;
  if (b == 0) return;
  const size_t NM = (size_t)N * M;
  u += b * n * n;
  if (sino != nullptr) sino += b * NM;
  if (ep.target != nullptr) ep.target += b * NM;
  if (ep.vb1 != nullptr) ep.vb1 += b * NM;
  if (ep.s1 != nullptr) ep.s1 += b * NM;
  if (ep.y1 != nullptr) ep.y1 += b * NM;
  if (ep.r != nullptr) ep.r += b * NM;
  if (ep.q1 != nullptr) ep.q1 += b * NM;
  if (ep.mask != nullptr) ep.mask += b * (size_t)N * ((M + 31) >> 5);
  if (ep.aux != nullptr) ep.aux += b * NM;
}

// Output of one projected bin: either the raw value R(u)[l][k], or the PDRQS1
// sinogram-side update (§4.4) with r = R(u)[l][k] / beta:
//   v1 = vb1 + sigma r, y1 = prox(2 v1 - vb1, sigma), vb1 <- vb1 + y1 - v1,
//   s1 = vb1 + sigma r  (mode 1: only s1 = vb1 + sigma r; mode 2: also y1, r).
__device__ inline void fp_output(float *__restrict__ sino, const SinoEpi &ep, int M, int l, int k,
                                 float raw) {
  const size_t o = (size_t)l * M + k;
  // every epilogue mode writes vb1 or s1; with neither the raw value is stored
  if (ep.vb1 == nullptr && ep.s1 == nullptr) {
    sino[o] = raw;
    return;
  }
  const float r = raw * ep.inv_beta;
  if (ep.mode == 5) {
    // PDRQS2: the data residual b - A u (D0 empty)
    ep.s1[o] = ep.target[o] - r;
    return;
  }
  const float vb = ep.vb1[o];
  if (ep.mode == 7 || ep.mode == 8) {
    // PDRQ3 (§4.4, table of splittings): off D0 the fit's quadratic part is
    // the dual's, vb1 <- (vb1 + sigma (r - b)) / (1 + sigma); on D0 the
    // constraint's resolvent as in PDRQS1.  The cache for the next u-step is
    // s1 = D (vb1 + sigma (r - g)), D = 1/(1 + sigma) and g = b off D0, D = 1
    // and g = 0 on D0.  Mode 8 writes only that cache.
    const int MW7 = (M + 31) >> 5;
    const bool d0 =
        ep.mask != nullptr && ((ep.mask[(size_t)l * MW7 + (k >> 5)] >> (k & 31)) & 1u);
    const float sg = ep.sigma, tg = ep.target[o];
    float nb = vb;
    if (ep.mode == 7) {
      if (d0) {
        const float v1 = fmaf(sg, r, vb);
        nb = vb + fminf(2.f * v1 - vb - sg * tg, 0.f) - v1;
      } else {
        nb = fmaf(sg, r - tg, vb) / (1.f + sg);
      }
      ep.vb1[o] = nb;
    }
    ep.s1[o] = d0 ? fmaf(sg, r, nb) : fmaf(sg, r - tg, nb) / (1.f + sg);
    return;
  }
  if (ep.mode == 6) {
    // ADMM z-step and multiplier update (§4.6), data block, mu in the sigma
    // field: s = A u + eta_w, w = (b + mu s)/(1 + mu), eta_w <- s - w, and
    // the next u-step's residual term (w - eta_w) - A u = 2 w - s - A u
    const float sw = r + vb;
    const float w = fmaf(ep.sigma, sw, ep.target[o]) / (1.f + ep.sigma);
    ep.vb1[o] = sw - w;
    ep.s1[o] = 2.f * w - sw - r;
    return;
  }
  if (ep.mode == 4) {
    // Algorithm CP: v <- resolvent of the data term's conjugate, step sigma,
    // at v + sigma A u (here u is the extrapolated iterate)
    const int MW4 = (M + 31) >> 5;
    const bool d0 =
        ep.mask != nullptr && ((ep.mask[(size_t)l * MW4 + (k >> 5)] >> (k & 31)) & 1u);
    const float qv = fmaf(ep.sigma, r, vb);
    const float tg = ep.target[o];
    ep.vb1[o] = d0 ? fminf(qv - ep.sigma * tg, 0.f) : (qv - ep.sigma * tg) / (1.f + ep.sigma);
    return;
  }
  if (ep.mode == 1) {
    ep.s1[o] = fmaf(ep.sigma, r, vb);
    return;
  }
  if (ep.mode == 3) {
    // reverse sweep of the unrolled iteration: with r = A x for the adjoint x
    // of u_tmp, S1 = -sigma r; vb1 holds Q1 (in), s1 receives the adjoint of
    // the previous vb1, Q1 + S1, and y1 the deferred sinogram term sigma S1.
    const float sb = -ep.sigma * r;
    ep.s1[o] = vb + sb;
    ep.y1[o] = ep.sigma * sb;
    return;
  }
  const int MW = (M + 31) >> 5;
  const bool on_d0 =
      ep.mask != nullptr && ((ep.mask[(size_t)l * MW + (k >> 5)] >> (k & 31)) & 1u);
  const float v1 = fmaf(ep.sigma, r, vb);
  const float q = 2.f * v1 - vb;
  if (ep.q1 != nullptr) ep.q1[o] = q;
  const float tg = ep.target[o];
  const float sg = ep.sigma;
  float y;
  if (ep.fit == 0) {
    y = on_d0 ? fminf(q - sg * tg, 0.f) : (q - sg * tg) / (1.f + sg);
  } else if (on_d0) {
    // data-term variants of §3.5 on D0: no term (ignore), the fit plus the
    // bound (everywhere: q - sigma max((q + b)/(1 + sigma), C~)), else the bound
    if (ep.fit == 2)
      y = 0.f;
    else if (ep.fit == 3)
      y = q - sg * fmaxf((q + ep.aux[o]) / (1.f + sg), tg);
    else
      y = fminf(q - sg * tg, 0.f);
  } else {
    // off D0: weighted fit (q - sigma b)/(1 + sigma/w), hard constraint q - sigma b
    if (ep.fit == 1)
      y = (q - sg * tg) / (1.f + sg / ep.aux[o]);
    else if (ep.fit == 4)
      y = q - sg * tg;
    else
      y = (q - sg * tg) / (1.f + sg);
  }
  const float nb = vb + y - v1;
  ep.vb1[o] = nb;
  ep.s1[o] = fmaf(ep.sigma, r, nb);
  if (ep.mode == 2) {
    ep.y1[o] = y;
    ep.r[o] = r;
  }
}

// Staging of one chunk of kFpRows walk rows x W columns (W <= kFpMaxWidth)
// for the forward projector: each of the kFpThreads threads loads
// kFpPrefetch pixels (zero outside the image).  Walk rows are image rows
// (tr = false: lanes run along the row) or image columns (tr = true: lanes run
// along q, which is contiguous in memory).
__device__ inline void fp_stage_load(float (&v)[kFpPrefetch], const float *__restrict__ u, int n,
                                     bool tr, bool fi, bool fo, int q0, int rows, int plo,
                                     int W) {
  const int t = threadIdx.x;
  if (!tr) {
#pragma unroll
    for (int mr = 0; mr < kFpRows / (kFpThreads / 64); ++mr) {
      const int r = (t >> 6) + (kFpThreads / 64) * mr;
      const int q = q0 + r;
      const float *urow = u + (size_t)(fo ? n - 1 - q : q) * n;
      const bool rok = r < rows;
#pragma unroll
      for (int mc = 0; mc < kFpMaxWidth / 64; ++mc) {
        const int c = (t & 63) + 64 * mc;
        const int p = plo + c;
        float x = 0.f;
        if (rok && c < W && (unsigned)p < (unsigned)n) x = urow[fi ? n - 1 - p : p];
        v[mr * (kFpMaxWidth / 64) + mc] = x;
      }
    }
  } else {
    const int r = t & (kFpRows - 1);
    const int q = q0 + r;
    const float *ucol = u + (fo ? n - 1 - q : q);
    const bool rok = r < rows;
#pragma unroll
    for (int m = 0; m < kFpPrefetch; ++m) {
      const int c = (t / kFpRows) + (kFpThreads / kFpRows) * m;
      const int p = plo + c;
      float x = 0.f;
      if (rok && c < W && (unsigned)p < (unsigned)n) x = ucol[(size_t)(fi ? n - 1 - p : p) * n];
      v[m] = x;
    }
  }
}

__device__ inline void fp_stage_store(const float (&v)[kFpPrefetch], float *tile, int ldw, bool tr,
                                      int rows, int W) {
  const int t = threadIdx.x;
  if (!tr) {
#pragma unroll
    for (int mr = 0; mr < kFpRows / (kFpThreads / 64); ++mr) {
      const int r = (t >> 6) + (kFpThreads / 64) * mr;
#pragma unroll
      for (int mc = 0; mc < kFpMaxWidth / 64; ++mc) {
        const int c = (t & 63) + 64 * mc;
        if (r < rows && c < W) tile[r * ldw + c] = v[mr * (kFpMaxWidth / 64) + mc];
      }
    }
  } else {
    const int r = t & (kFpRows - 1);
#pragma unroll
    for (int m = 0; m < kFpPrefetch; ++m) {
      const int c = (t / kFpRows) + (kFpThreads / kFpRows) * m;
      if (r < rows && c < W) tile[r * ldw + c] = v[m];
    }
  }
}

// One row of the walk for a strip: e = t(ps) - k 2^30 in [0, A); one row
// down, e += B, and when that reaches A the strip starts one pixel earlier.
__device__ inline void walk_row(uint32_t &e, int &ps, uint32_t A, uint32_t B) {
  const uint32_t en = e + B;
  uint32_t d;
  const bool below = __builtin_sub_overflow(en, A, &d);  // en < A
  e = below ? en : d;
  ps = ps - 1 + (below ? 1 : 0);
}

// The same step on a pointer into the staged rows (row pitch `stride`).
__device__ inline void walk_row_ptr(uint32_t &e, const float *&pt, uint32_t A, uint32_t B,
                                    int stride) {
  const uint32_t en = e + B;
  uint32_t d;
  const bool below = __builtin_sub_overflow(en, A, &d);  // en < A
  e = below ? en : d;
  pt += (stride - 1) + (int)below;  // one add with the borrow as carry-in
}

template <bool CHECK_FIRST>
__global__ __launch_bounds__(kFpThreads) void k_radon_fwd(
    const float *__restrict__ u, int n, int M, const FpAngle *__restrict__ angs,
    const FpGroup *__restrict__ groups, const int2 *__restrict__ regions,
    const int2 *__restrict__ chunk_range, const int2 *__restrict__ work, int n_chunks, int ldw,
    float *__restrict__ sino, SinoEpi ep, int N) {
  extern __shared__ float tile[];  // 2 x kFpRows * ldw
  fp_batch_offsets(u, sino, ep, n, N, M);
  const int2 wk = work[blockIdx.x];  // (group, block along the bins)
  const FpGroup grp = groups[wk.x];
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int blk = wk.y;
  const int nblk_eff = grp.nblk > 0 ? grp.nblk : 1;

  // Bins no pixel reaches hold zero (block 0 below kmin, last block above kmax).
  if (blk == 0) {
    const int lim = min(grp.kmin, M);
    for (int a = 0; a < grp.count; ++a) {
      const int l = angs[grp.first + a].l;
      for (int k = threadIdx.x; k < lim; k += blockDim.x) fp_output(sino, ep, M, l, k, 0.f);
    }
  }
  if (blk == nblk_eff - 1) {
    const int from = max(grp.kmax + 1, grp.kmin);
    for (int a = 0; a < grp.count; ++a) {
      const int l = angs[grp.first + a].l;
      for (int k = max(from, 0) + threadIdx.x; k < M; k += blockDim.x)
        fp_output(sino, ep, M, l, k, 0.f);
    }
  }
  if (blk >= grp.nblk) return;

  const int kb = grp.kmin + blk * (kFpStrips - 1);  // first output bin
  const int k = kb - 1 + lane;                      // this lane's strip
  const uint32_t one = 1u << kFixBits;
  // chunks in which some strip of this block meets the image (host-computed)
  const int2 crange = chunk_range[grp.range + blk];
  const int ch_first = crange.x, ch_last = crange.y;
  const int q_first = ch_first * kFpRows;

  // Walk state per angle slot.  Inactive slots (beyond the group's count)
  // walk a harmless empty strip: their results are never stored.
  // P = sum u, Q = sum (e1 2^-30 ... in units of 2^-30) over the strip's first
  // pixels and second pixels' shared part, Q2 = sum of second pixels (whose
  // fraction is e1 + A).
  uint32_t e[kFpPerThread], A[kFpPerThread], B[kFpPerThread], lim2[kFpPerThread];
  int ps[kFpPerThread];
  float P[kFpPerThread], Q[kFpPerThread], Q2[kFpPerThread];
#pragma unroll
  for (int g = 0; g < kFpPerThread; ++g) {
    const int slot = wave * kFpPerThread + g;
    P[g] = 0.f;
    Q[g] = 0.f;
    Q2[g] = 0.f;
    e[g] = 0u;
    ps[g] = -(1 << 29);
    A[g] = one;
    B[g] = 0u;
    if (slot < grp.count) {
      const FpAngle fa = angs[grp.first + slot];
      A[g] = fa.A;
      B[g] = fa.B;
      const int64_t num = (int64_t)k * ((int64_t)1 << kFixBits) - fa.T -
                          (int64_t)q_first * (int64_t)fa.B;
      int64_t pp = (int64_t)ceil((double)num / (double)fa.A);
      int64_t ee = pp * (int64_t)fa.A - num;
      if (ee < 0) {
        pp += 1;
        ee += fa.A;
      } else if (ee >= (int64_t)fa.A) {
        pp -= 1;
        ee -= fa.A;
      }
      pp = pp < -(1 << 29) ? -(1 << 29) : (pp > (1 << 29) ? (1 << 29) : pp);
      ps[g] = (int)pp;
      e[g] = (uint32_t)ee;
    }
    // the second pixel (fraction e + A) is in the strip iff e < 2^30 - A
    lim2[g] = A[g] < one ? one - A[g] : 0u;
  }

  const int2 *reg = regions + grp.region + blk * n_chunks;
  const bool tr = (grp.cls & 1) != 0;
  const bool fi = (grp.cls & 2) != 0;
  const bool fo = (grp.cls & 4) != 0;
  constexpr int RB = 8;  // rows whose LDS reads are issued together

  // Staged image rows are double-buffered; the next chunk's pixels are
  // loaded into registers while the current chunk is walked.
  float pf[kFpPrefetch];
  int2 rg_next = make_int2(0, 4);
  if (ch_first <= ch_last) {
    rg_next = reg[ch_first];
    fp_stage_load(pf, u, n, tr, fi, fo, q_first, min(kFpRows, n - q_first), rg_next.x, rg_next.y);
  }
  for (int ch = ch_first; ch <= ch_last; ++ch) {
    const int q0 = ch * kFpRows;
    const int rows = min(kFpRows, n - q0);
    const int2 rg = rg_next;
    const int plo = rg.x, W = rg.y;
    float *buf = tile + ((ch - ch_first) & 1) * (kFpRows * ldw);
    fp_stage_store(pf, buf, ldw, tr, rows, W);
    __syncthreads();
    if (ch + 1 <= ch_last) {
      rg_next = reg[ch + 1];
      const int q1 = q0 + kFpRows;
      fp_stage_load(pf, u, n, tr, fi, fo, q1, min(kFpRows, n - q1), rg_next.x, rg_next.y);
    }
    const float *tile_c = buf;
    // The strip's first pixel ps, clamped to [-2, n] (zero-staged columns
    // outside the image), addresses the staged row at byte offset
    // 4 (r ldw + ps - plo).
    const int cneg = -2, cpos = n;
    int r0 = 0;
    for (; r0 + RB <= rows; r0 += RB) {
      uint32_t off[RB][kFpPerThread], ev[RB][kFpPerThread];
      // 1. the walk: positions and fractions of RB rows (independent of the data)
#pragma unroll
      for (int r = 0; r < RB; ++r) {
        const int rowbase = ((r0 + r) * ldw - plo) * 4;
#pragma unroll
        for (int g = 0; g < kFpPerThread; ++g) {
          off[r][g] = (uint32_t)(med3i(ps[g], cneg, cpos) * 4 + rowbase);
          ev[r][g] = e[g];
          walk_row(e[g], ps[g], A[g], B[g]);
        }
      }
      // 2. all LDS reads of the batch
      float u1[RB][kFpPerThread], u2[RB][kFpPerThread];
#pragma unroll
      for (int r = 0; r < RB; ++r) {
#pragma unroll
        for (int g = 0; g < kFpPerThread; ++g) {
          const float *pt = reinterpret_cast<const float *>(
              reinterpret_cast<const char *>(tile_c) + off[r][g]);
          u1[r][g] = pt[0];
          u2[r][g] = pt[1];
        }
      }
      // 3. accumulate: first pixel (fraction e), second pixel (e + A) if in the strip
#pragma unroll
      for (int r = 0; r < RB; ++r) {
#pragma unroll
        for (int g = 0; g < kFpPerThread; ++g) {
          const uint32_t e1 = ev[r][g];
          float a1 = u1[r][g];
          if (CHECK_FIRST) a1 = (e1 < one) ? a1 : 0.f;
          const float a2 = (e1 < lim2[g]) ? u2[r][g] : 0.f;
          const float sum = a1 + a2;
          P[g] += sum;
          Q[g] = fmaf((float)e1, sum, Q[g]);
          Q2[g] += a2;
        }
      }
    }
    for (int r = r0; r < rows; ++r) {  // ragged last chunk
#pragma unroll
      for (int g = 0; g < kFpPerThread; ++g) {
        const int c = med3i(ps[g], cneg, cpos) - plo;
        const float *trow = tile_c + r * ldw;
        const uint32_t e1 = e[g];
        float a1 = trow[c];
        if (CHECK_FIRST) a1 = (e1 < one) ? a1 : 0.f;
        const float a2 = (e1 < lim2[g]) ? trow[c + 1] : 0.f;
        const float sum = a1 + a2;
        P[g] += sum;
        Q[g] = fmaf((float)e1, sum, Q[g]);
        Q2[g] += a2;
        walk_row(e[g], ps[g], A[g], B[g]);
      }
    }
  }

  const float inv = 1.0f / (float)one;
#pragma unroll
  for (int g = 0; g < kFpPerThread; ++g) {
    const int slot = wave * kFpPerThread + g;
    const float qt = fmaf((float)A[g], Q2[g], Q[g]);  // sum of fraction * u, in 2^-30 units
    const float qprev = __shfl_up(qt, 1, 64);
    if (slot < grp.count && lane >= 1 && k <= grp.kmax && k < M) {
      const int l = angs[grp.first + slot].l;
      fp_output(sino, ep, M, l, k, fmaf(qprev - qt, inv, P[g]));
    }
  }
}

// ---------------------------------------------------------------------------
// R_h for SL angles that share one walk (SL = 2: pairs).  With equispaced
// angles theta, pi/2 - theta, pi - theta and pi/2 + theta have identical walk
// constants (T, A, B) and differ only in how (p, q) maps to image pixels.
// (Four angles per walk were measured slower on gfx950: half as many waves
// to hide LDS latency, and twice the staging per wave.)  The strips and the
// output are those of k_radon_fwd, the walk a 64-bit fixed-point one
// (walk_y0): its high word addresses the staged pixel, its low word is the
// interpolation fraction, and a row costs one add.  The SL angles of a set
// walk the same positions; a wave owns two sets (pairs A and B) of 32
// strips, interleaved in groups of 16 lanes (pr_strip, pr_pair), and a
// workgroup MultiCfg<SL>::kWaves waves over one block of kPrStrips strips.  Each chunk stages the same
// (row, column) window SL times -- once per angle, through that angle's
// transpose/mirror mapping -- as rows of pitch kLdw, the SL copies of a row
// adjacent, so that the reads of all SL angles at (row, ps) share addresses.
// Strip positions are not clamped: the host-computed windows cover every
// position the block's lanes reach, with zeros outside the image.
template <int SL>
struct MultiCfg;
template <>
struct MultiCfg<2> {
  static constexpr int kWaves = kPrWaves, kRows = kFpRows;
};
template <>
struct MultiCfg<4> {
  static constexpr int kWaves = kQuadWaves, kRows = kFpRows;
};

constexpr int kMultiWidth = 128;              // staged columns per chunk
// LDS buffers of staged rows: with 2, chunk c + 1 is stored while chunk c is
// read (one barrier per chunk); with 1, a second barrier per chunk, half the
// LDS and so more resident workgroups.
constexpr int kFpMultiBufs = 1;
constexpr int kLdw = kMultiWidth + 1;         // LDS row pitch (floats)

// Buffer loads with range checking (a load whose byte offset is not below
// the descriptor's record count returns 0, a documented property of buffer
// addressing) provide the zeros outside the image, so staging has no
// branches and no masks: in the row case each wave reads one image row
// through a descriptor covering just that row; in the column case one
// descriptor covers the image and an offset outside it comes from a column
// index outside [0, n).  Positions beyond the window or past the chunk's
// last row are staged too but never read.

template <int SL>
struct Stage {
  static constexpr int kWaves = MultiCfg<SL>::kWaves, kRows = MultiCfg<SL>::kRows;
  static constexpr int kThreads = 64 * kWaves;
  static constexpr int kPer = kRows * kMultiWidth / kThreads;  // values per thread per tile

  __device__ static void load(float (&v)[kPer], const float *__restrict__ u, int n, int cls,
                              int q0, int rows, int plo) {
    const bool tr = (cls & 1) != 0, fi = (cls & 2) != 0, fo = (cls & 4) != 0;
    const int t = threadIdx.x;
    if (!tr) {
      // the wave index in a scalar register, so that the descriptor is one too
      const int wv = __builtin_amdgcn_readfirstlane(t >> 6);
      // byte offset of column p0 = plo + lane; position p0 + 64 mc is 64
      // columns further along the (possibly mirrored) row; the same offsets
      // serve every row (each row has its own descriptor)
      int off[kMultiWidth / 64];
      {
        const int p0 = plo + (t & 63);
        const int o0 = (fi ? n - 1 - p0 : p0) * 4;
        const int dstep = fi ? -256 : 256;
#pragma unroll
        for (int mc = 0; mc < kMultiWidth / 64; ++mc) off[mc] = own_offset(o0 + mc * dstep);
      }
#pragma unroll
      for (int mr = 0; mr < kRows / kWaves; ++mr) {
        const int r = wv + kWaves * mr;  // wave-uniform
        const int q = min(q0 + r, n - 1);
        const float *urow = u + (size_t)(fo ? n - 1 - q : q) * n;
        const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
            (void *)urow, (short)0, r < rows ? n * 4 : 0, kBufWord3);
#pragma unroll
        for (int mc = 0; mc < kMultiWidth / 64; ++mc)
          v[mr * (kMultiWidth / 64) + mc] =
              __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, off[mc], 0, 0));
      }
    } else {
      const int r = t & (kRows - 1);
      const int q = min(q0 + r, n - 1);
      const int qi = fo ? n - 1 - q : q;
      const __amdgpu_buffer_rsrc_t rs =
          __builtin_amdgcn_make_buffer_rsrc((void *)u, (short)0, n * n * 4, kBufWord3);
      // image row of position p0 = plo + t / kRows; each further value is
      // kThreads / kRows rows on (up, when mirrored), a fixed byte step
      const int p0 = plo + t / kRows;
      const int o0 = ((fi ? n - 1 - p0 : p0) * n + qi) * 4;
      const int dstep = (fi ? -4 : 4) * (kThreads / kRows) * n;
      // a chain of offsets: each load takes its register as it is, one add apart
      int o = o0;
#pragma unroll
      for (int m = 0; m < kPer; ++m) {
        o = own_offset(o);
        v[m] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, o, 0, 0));
        o += dstep;
      }
    }
  }

  // Row r of angle `slot` starts at tile + (SL r + slot) kLdw; every staged
  // position is written (window positions beyond W too), so stores need no mask.
  __device__ static void store(const float (&v)[kPer], float *tile, int cls, int slot) {
    const int t = threadIdx.x;
    if (!(cls & 1)) {
#pragma unroll
      for (int mr = 0; mr < kRows / kWaves; ++mr) {
        const int r = (t >> 6) + kWaves * mr;
#pragma unroll
        for (int mc = 0; mc < kMultiWidth / 64; ++mc) {
          const int c = (t & 63) + 64 * mc;
          tile[(SL * r + slot) * kLdw + c] = v[mr * (kMultiWidth / 64) + mc];
        }
      }
    } else {
      const int r = t & (kRows - 1);
#pragma unroll
      for (int m = 0; m < kPer; ++m) {
        const int c = (t / kRows) + (kThreads / kRows) * m;
        tile[(SL * r + slot) * kLdw + c] = v[m];
      }
    }
  }
};

// Accumulation of one staged row for one angle: first pixel (fraction e),
// second pixel (fraction e + A) when it lies in the strip.
template <bool CHECK_FIRST>
__device__ inline void acc_row(float x1, float x2, bool in1, bool in2, float ef, float &P,
                               float &Q, float &S) {
  const float a0 = CHECK_FIRST ? (in1 ? x1 : 0.f) : x1;
  const float a2 = in2 ? x2 : 0.f;
  const float sa = a0 + a2;
  P += sa;
  Q = fmaf(ef, sa, Q);
  S += a2;
}

// The same with the second pixel already zero when it lies outside the strip
// (read from a zero slot instead of the staged row).
template <bool CHECK_FIRST>
__device__ inline void acc_row_z(float x1, float a2, bool in1, float ef, float &P, float &Q,
                                 float &S) {
  const float a0 = CHECK_FIRST ? (in1 ? x1 : 0.f) : x1;
  const float sa = a0 + a2;
  P += sa;
  Q = fmaf(ef, sa, Q);
  S += a2;
}

// TVF: the launch also holds the gradient-side update's workgroups (a
// separate instantiation, so that traces tell the two launches apart).
template <int SL, bool CHECK_FIRST, bool TVF>
__global__ __launch_bounds__(64 * MultiCfg<SL>::kWaves) void k_radon_fwd_multi(
    const float *__restrict__ u, int n, int M, const FpAngle *__restrict__ angs,
    const FpGroup *__restrict__ groups, const int2 *__restrict__ regions,
    const int2 *__restrict__ chunk_range, const int2 *__restrict__ work, int n_chunks,
    float *__restrict__ sino, SinoEpi ep, int N, int n_work, TvArgs tv) {
  if (TVF && (int)blockIdx.x >= n_work) {
    // workgroups past the projection's run the gradient-side update (rows
    // b, b + tv.blocks, ...): memory-bound work next to the ALU-bound walk
    for (int j = (int)blockIdx.x - n_work; j < tv.n; j += tv.blocks)
      for (int i = threadIdx.x; i < tv.n; i += blockDim.x) tv_update_px(tv, i, j, blockIdx.z);
    return;
  }
  using St = Stage<SL>;
  constexpr int kRows = St::kRows;
  constexpr int kStride = SL * kLdw;  // staged row pitch (floats)
  __shared__ float tile[kFpMultiBufs * kRows * kStride];  // buffers x kRows x SL angles x kLdw
  // zero slot: a second pixel outside the strip is read from zs + 1 + s kLdw
  __shared__ float zs[kStride + 1];
  for (int t = threadIdx.x; t < kStride + 1; t += blockDim.x) zs[t] = 0.f;  // before 1st barrier
  fp_batch_offsets(u, sino, ep, n, N, M);
  const int2 wk = work[blockIdx.x];  // (group, block along the bins)
  const FpGroup grp = groups[wk.x];
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int lane = threadIdx.x & 63;
  const int so = pr_strip(lane);              // strip offset in the block
  const int item = 2 * wave + pr_pair(lane);  // this lane's pair in the group
  const int blk = wk.y;
  const int nblk_eff = grp.nblk > 0 ? grp.nblk : 1;
  const FpAngle *pa = angs + SL * grp.first;
  int cls[SL];
#pragma unroll
  for (int s = 0; s < SL; ++s) cls[s] = (grp.clss >> (8 * s)) & 0xff;

  // Bins no pixel reaches hold zero (block 0 below kmin, last block above kmax).
  if (blk == 0) {
    const int lim = min(grp.kmin, M);
    for (int a = 0; a < SL * grp.count; ++a) {
      const int l = pa[a].l;
      if (l < 0) continue;
      for (int k = threadIdx.x; k < lim; k += blockDim.x) fp_output(sino, ep, M, l, k, 0.f);
    }
  }
  if (blk == nblk_eff - 1) {
    const int from = max(max(grp.kmax + 1, grp.kmin), 0);
    for (int a = 0; a < SL * grp.count; ++a) {
      const int l = pa[a].l;
      if (l < 0) continue;
      for (int k = from + threadIdx.x; k < M; k += blockDim.x) fp_output(sino, ep, M, l, k, 0.f);
    }
  }
  if (blk >= grp.nblk) return;

  const int kb = grp.kmin + blk * (kPrStrips - 1);  // first output bin
  const int k = kb - 1 + so;                        // this lane's strip
  const uint32_t one = 1u << kFixBits;
  const int2 crange = chunk_range[grp.range + blk];
  const int ch_first = crange.x, ch_last = crange.y;
  const int q_first = ch_first * kRows;
  const bool active = item < grp.count;

  // Lane state: the 64-bit fixed-point position y of the strip's first
  // pixel (walk_y0), its high word relative to the staged window while a
  // chunk is processed.  Neighbouring strips differ by exactly dfix, so a
  // strip's last pixel is always the pixel before the next strip's first
  // one.  A strip holds one or two pixels when dfix >= 2^32 (the second one
  // iff the fraction lies above ~lo(dfix)), else none or one (the first one
  // iff the fraction is at least 2^32 - dfix).
  uint64_t y = 0, E = 0;
  uint32_t L1 = 0u, L2 = 0xffffffffu;
  float a30 = 0.f;
  if (active) {
    const FpAngle fa = pa[SL * item];
    a30 = (float)fa.A * (1.0f / (float)one);
    E = ((uint64_t)kStride << 32) - fa.dlt;
    y = walk_y0(kb - 1, q_first, fa.T, fa.A, fa.B) + (uint64_t)so * fa.dfix;
    const uint32_t dlo = (uint32_t)fa.dfix;
    if ((fa.dfix >> 32) != 0) {
      L2 = ~dlo;
    } else {
      L1 = 0u - dlo;
    }
  }
  float P[SL], G[SL], S[SL];
#pragma unroll
  for (int s = 0; s < SL; ++s) P[s] = G[s] = S[s] = 0.f;

  const int2 *reg = regions + grp.region + blk * n_chunks;
  constexpr int RB = 16;  // rows whose LDS reads are issued together
  float pf[SL][St::kPer];
  int2 rg_next = make_int2(0, 4);
  if (ch_first <= ch_last) {
    rg_next = reg[ch_first];
    const int rows0 = min(kRows, n - q_first);
#pragma unroll
    for (int s = 0; s < SL; ++s) St::load(pf[s], u, n, cls[s], q_first, rows0, rg_next.x);
  }
  for (int ch = ch_first; ch <= ch_last; ++ch) {
    const int q0 = ch * kRows;
    const int rows = min(kRows, n - q0);
    const int plo = rg_next.x;
    float *buf = tile + ((ch - ch_first) % kFpMultiBufs) * (kRows * kStride);
    // one buffer: every wave must be done with the previous chunk first
    if (kFpMultiBufs == 1 && ch > ch_first) __syncthreads();
#pragma unroll
    for (int s = 0; s < SL; ++s) St::store(pf[s], buf, cls[s], s);
    __syncthreads();
    if (ch + 1 <= ch_last) {
      rg_next = reg[ch + 1];
      const int q1 = q0 + kRows;
      const int rows1 = min(kRows, n - q1);
#pragma unroll
      for (int s = 0; s < SL; ++s) St::load(pf[s], u, n, cls[s], q1, rows1, rg_next.x);
    }
    if (active) {
      // high word: index into the staged rows (row r of the window starts at
      // buf + r kStride, and E moves one row down and B / A pixels left)
      uint64_t yc = y - ((uint64_t)(int64_t)plo << 32);
      int r0 = 0;
      for (; r0 + RB <= rows; r0 += RB) {
        const float *pr[RB], *pr2[RB];
        uint32_t lo[RB];
#pragma unroll
        for (int r = 0; r < RB; ++r) {
          const float *pt = buf + (int32_t)(yc >> 32);
          lo[r] = (uint32_t)yc;
          pr[r] = (!CHECK_FIRST || lo[r] >= L1) ? pt : zs;
          // the second pixels of all SL angles come from the row or the zero slot
          pr2[r] = lo[r] > L2 ? pt : zs;
          yc += E;
          // keep the walk one 64-bit add per row (not 16 running offsets)
          asm("" : "+v"(yc));
        }
        float x1[RB][SL], x2[RB][SL];
#pragma unroll
        for (int r = 0; r < RB; ++r) {
#pragma unroll
          for (int s = 0; s < SL; ++s) {
            x1[r][s] = pr[r][s * kLdw];
            x2[r][s] = pr2[r][s * kLdw + 1];
          }
        }
#pragma unroll
        for (int r = 0; r < RB; ++r) {
          const float gf = (float)lo[r];
#pragma unroll
          for (int s = 0; s < SL; ++s) {
            const float sa = x1[r][s] + x2[r][s];
            P[s] += sa;
            G[s] = fmaf(gf, sa, G[s]);
            S[s] += x2[r][s];
          }
        }
      }
      for (int r = r0; r < rows; ++r) {  // ragged last chunk
        const float *pt = buf + (int32_t)(yc >> 32);
        const uint32_t l0 = (uint32_t)yc;
        const float *p1 = (!CHECK_FIRST || l0 >= L1) ? pt : zs;
        const float *p2 = l0 > L2 ? pt : zs;
        const float gf = (float)l0;
#pragma unroll
        for (int s = 0; s < SL; ++s) {
          const float x1 = p1[s * kLdw], x2 = p2[s * kLdw + 1];
          const float sa = x1 + x2;
          P[s] += sa;
          G[s] = fmaf(gf, sa, G[s]);
          S[s] += x2;
        }
        yc += E;
      }
      y = yc + ((uint64_t)(int64_t)(plo - rows * kStride) << 32);
    }
  }

  // the strip's fraction-weighted sum: its pixels lie 1 - g and 2 - g pixel
  // widths past the strip's start, i.e. A (1 - g) and A (2 - g) bin widths
  // in 2^-30 units, with g = lo 2^-32; the previous strip of the same pair
  // is one lane down, or 17 for strip 16
  float qt[SL], qp[SL];
  const int src = lane - (so == 16 ? 17 : 1);
#pragma unroll
  for (int s = 0; s < SL; ++s) {
    qt[s] = a30 * fmaf(G[s], -2.3283064365386963e-10f, P[s] + S[s]);
    qp[s] = __shfl(qt[s], src < 0 ? 0 : src, 64);
  }
  if (active && so >= 1 && k <= grp.kmax && k < M) {
#pragma unroll
    for (int s = 0; s < SL; ++s) {
      const int l = pa[SL * item + s].l;
      if (l >= 0) fp_output(sino, ep, M, l, k, P[s] + (qp[s] - qt[s]));
    }
  }
}

int launch_radon_fwd(const ct_plan *p, const float *u, float *out, hipStream_t s,
                     const SinoEpi *epi, int nb, const TvArgs *tv, bool *fused) {
  SinoEpi ep{};
  if (epi) ep = *epi;
  const int N = p->g.n_angles;
  dim3 grid(p->n_work, 1, nb);
  if (fused) *fused = false;
  if (p->slots == 2 || p->slots == 4) {
    const dim3 block(64 * (p->slots == 4 ? MultiCfg<4>::kWaves : MultiCfg<2>::kWaves));
    TvArgs ta{};
    if (tv != nullptr && tv->blocks > 0) {
      ta = *tv;
      grid.x += ta.blocks;
      if (fused) *fused = true;
    }
    auto go = [&](auto cf, auto tvf) {
      constexpr bool CF = decltype(cf)::value, TVF = decltype(tvf)::value;
      if (p->slots == 4)
        hipLaunchKernelGGL((k_radon_fwd_multi<4, CF, TVF>), grid, block, 0, s, u, p->g.n,
                           p->g.n_bins, p->d_fp, p->d_groups, p->d_regions, p->d_chunk_range,
                           p->d_work, p->n_chunks, out, ep, N, p->n_work, ta);
      else
        hipLaunchKernelGGL((k_radon_fwd_multi<2, CF, TVF>), grid, block, 0, s, u, p->g.n,
                           p->g.n_bins, p->d_fp, p->d_groups, p->d_regions, p->d_chunk_range,
                           p->d_work, p->n_chunks, out, ep, N, p->n_work, ta);
    };
    const bool with_tv = ta.blocks > 0;
    if (p->check_first) {
      if (with_tv)
        go(std::true_type{}, std::true_type{});
      else
        go(std::true_type{}, std::false_type{});
    } else {
      if (with_tv)
        go(std::false_type{}, std::true_type{});
      else
        go(std::false_type{}, std::false_type{});
    }
    CT_TRY_HIP(hipGetLastError());
    return CT_OK;
  }
  const int ldw = (p->wmax % 2 == 0) ? p->wmax + 1 : p->wmax;
  const size_t lds = 2 * sizeof(float) * kFpRows * ldw;
  if (p->check_first)
    hipLaunchKernelGGL(k_radon_fwd<true>, grid, dim3(kFpThreads), lds, s, u, p->g.n, p->g.n_bins,
                       p->d_fp, p->d_groups, p->d_regions, p->d_chunk_range, p->d_work, p->n_chunks, ldw,
                       out, ep, N);
  else
    hipLaunchKernelGGL(k_radon_fwd<false>, grid, dim3(kFpThreads), lds, s, u, p->g.n, p->g.n_bins,
                       p->d_fp, p->d_groups, p->d_regions, p->d_chunk_range, p->d_work, p->n_chunks, ldw,
                       out, ep, N);
  CT_TRY_HIP(hipGetLastError());
  return CT_OK;
}

}  // namespace ctpd
