// Discrete Radon pair R_h / R_h^* on gfx950 (thesis §3.1).
//
// Both kernels evaluate the bin coordinate of pixel (i, j) at angle l,
//   t = (x_i cos theta_l + y_j sin theta_l)/ds + (M-1)/2,
// from constants quantized to multiples of 2^-30, so t itself is an exact
// multiple of 2^-30: the backprojection evaluates it exactly in FP64, the
// forward projection exactly in integers.  The interpolation weight
// alpha = t - floor(t) is rounded once to FP32 in both, giving bit-identical
// weights; R_h is the transpose of R_h^* up to FP32 summation order.
#include "common.hpp"

namespace ctpd {

// ---------------------------------------------------------------------------
// R_h^*: pixel-driven gather.  One workgroup per 16x16 pixel tile, one pixel
// per thread.  Angles are processed in chunks; for every angle of a chunk the
// detector segment the tile projects onto is staged in LDS as pairs
// (v[k], v[k+1] - v[k]) so that one 8-byte LDS read and one FMA interpolate.
// Epilogue: out = c1 * R^*(v) + c2 * div_h(p) (p optional; §3.1 divergence).
__global__ __launch_bounds__(256) void k_radon_adj(
    const float *__restrict__ sino, int n, int N, int M, const BpAngle *__restrict__ ang,
    int seg, const float *__restrict__ pfield, float c1, float c2, float inv_h,
    float *__restrict__ out) {
  extern __shared__ float2 vd[];  // kBpChunk * seg
  __shared__ int kmin_s[kBpChunk];
  __shared__ int row_s[kBpChunk];
  const int tx = threadIdx.x & (kBpTile - 1);
  const int ty = threadIdx.x / kBpTile;
  const int i0 = blockIdx.x * kBpTile, j0 = blockIdx.y * kBpTile;
  const int i = i0 + tx, j = j0 + ty;
  const bool inside = (i < n) && (j < n);
  const double di = (double)i, dj = (double)j;
  float acc_v = 0.f, acc_d = 0.f;

  for (int c0 = 0; c0 < N; c0 += kBpChunk) {
    const int nc = min(kBpChunk, N - c0);
    __syncthreads();
    if ((int)threadIdx.x < nc) {
      const BpAngle A = ang[c0 + threadIdx.x];
      const double ic = (A.a >= 0.0) ? (double)i0 : (double)(i0 + kBpTile - 1);
      const double jc = (A.b >= 0.0) ? (double)j0 : (double)(j0 + kBpTile - 1);
      const double tmin = fma(jc, A.b, fma(ic, A.a, A.t0));
      kmin_s[threadIdx.x] = (int)floor(tmin);
      row_s[threadIdx.x] = A.l;
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < nc * seg; idx += blockDim.x) {
      const int c = idx / seg;
      const int e = idx - c * seg;
      const int k = kmin_s[c] + e;
      const float *row = sino + (size_t)row_s[c] * M;
      const float v0 = (k >= 0 && k < M) ? row[k] : 0.f;
      const float v1 = (k + 1 >= 0 && k + 1 < M) ? row[k + 1] : 0.f;
      vd[idx] = make_float2(v0, v1 - v0);
    }
    __syncthreads();
    if (inside) {
      for (int c = 0; c < nc; ++c) {
        const BpAngle A = ang[c0 + c];
        const double t = fma(dj, A.b, fma(di, A.a, A.t0));  // exact
        const double fl = floor(t);
        const int kk = min(max((int)fl - kmin_s[c], 0), seg - 1);
        const float al = (float)(t - fl);                     // one rounding
        const float2 p = vd[c * seg + kk];
        acc_v += p.x;
        acc_d = fmaf(al, p.y, acc_d);
      }
    }
  }
  if (!inside) return;
  float res = c1 * (acc_v + acc_d);
  if (pfield != nullptr) {
    const float *p1 = pfield;
    const float *p2 = pfield + (size_t)n * n;
    const size_t o = (size_t)j * n + i;
    const float d1 = (i < n - 1 ? p1[o] : 0.f) - (i > 0 ? p1[o - 1] : 0.f);
    const float d2 = (j < n - 1 ? p2[o] : 0.f) - (j > 0 ? p2[o - n] : 0.f);
    res = fmaf(c2 * inv_h, d1 + d2, res);
  }
  out[(size_t)j * n + i] = res;
}

int launch_radon_adj(const ct_plan *p, const float *v, const float *pfield, float c1,
                     float c2, float *out, hipStream_t s) {
  const int n = p->g.n;
  dim3 grid((n + kBpTile - 1) / kBpTile, (n + kBpTile - 1) / kBpTile);
  const size_t lds = sizeof(float2) * kBpChunk * p->seg;
  hipLaunchKernelGGL(k_radon_adj, grid, dim3(256), lds, s, v, n, p->g.n_angles,
                     p->g.n_bins, p->d_bp, p->seg, pfield, c1, c2, (float)(1.0 / p->g.h),
                     out);
  CT_TRY_HIP(hipGetLastError());
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
__global__ __launch_bounds__(256) void k_radon_fwd(
    const float *__restrict__ u, int n, int M, const FpAngle *__restrict__ angs,
    const FpGroup *__restrict__ groups, const int2 *__restrict__ regions, int n_chunks,
    int ldw, int check_first, float *__restrict__ sino) {
  extern __shared__ float tile[];  // kFpRows * ldw
  const FpGroup grp = groups[blockIdx.x];
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int blk = blockIdx.y;
  const int nblk_eff = grp.nblk > 0 ? grp.nblk : 1;

  // Bins no pixel reaches are written as zero (block 0 below kmin, last block above kmax).
  if (blk == 0) {
    const int lim = min(grp.kmin, M);
    for (int a = 0; a < grp.count; ++a) {
      float *row = sino + (size_t)angs[grp.first + a].l * M;
      for (int k = threadIdx.x; k < lim; k += blockDim.x) row[k] = 0.f;
    }
  }
  if (blk == nblk_eff - 1) {
    const int from = max(grp.kmax + 1, grp.kmin);
    for (int a = 0; a < grp.count; ++a) {
      float *row = sino + (size_t)angs[grp.first + a].l * M;
      for (int k = max(from, 0) + threadIdx.x; k < M; k += blockDim.x) row[k] = 0.f;
    }
  }
  if (blk >= grp.nblk) return;

  const int kb = grp.kmin + blk * (kFpStrips - 1);  // first output bin
  const int k = kb - 1 + lane;                      // this lane's strip

  uint32_t e[kFpPerThread], A[kFpPerThread], B[kFpPerThread];
  int ps[kFpPerThread];
  float P[kFpPerThread], Q[kFpPerThread];
  int lrow[kFpPerThread];
  bool act[kFpPerThread];
#pragma unroll
  for (int g = 0; g < kFpPerThread; ++g) {
    const int slot = wave * kFpPerThread + g;
    act[g] = slot < grp.count;
    P[g] = 0.f;
    Q[g] = 0.f;
    e[g] = 0u;
    ps[g] = 0;
    A[g] = 1u;
    B[g] = 0u;
    lrow[g] = 0;
    if (act[g]) {
      const FpAngle fa = angs[grp.first + slot];
      A[g] = fa.A;
      B[g] = fa.B;
      lrow[g] = fa.l;
      const int64_t num = (int64_t)k * ((int64_t)1 << kFixBits) - fa.T;
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
  }

  const int2 *reg = regions + grp.region + blk * n_chunks;
  const bool tr = (grp.cls & 1) != 0;
  const bool fi = (grp.cls & 2) != 0;
  const bool fo = (grp.cls & 4) != 0;
  const uint32_t one = 1u << kFixBits;

  for (int ch = 0; ch < n_chunks; ++ch) {
    const int q0 = ch * kFpRows;
    const int rows = min(kFpRows, n - q0);
    const int2 rg = reg[ch];
    const int plo = rg.x, W = rg.y;
    __syncthreads();
    if (!tr) {
      // walk rows are image rows: consecutive lanes read consecutive pixels
      for (int r = wave; r < rows; r += kFpWaves) {
        const int q = q0 + r;
        const int jj = fo ? n - 1 - q : q;
        const float *urow = u + (size_t)jj * n;
        for (int c = lane; c < W; c += 64) {
          const int p = plo + c;
          float v = 0.f;
          if (p >= 0 && p < n) v = urow[fi ? n - 1 - p : p];
          tile[r * ldw + c] = v;
        }
      }
    } else {
      // walk rows are image columns: lanes run along q (contiguous in memory)
      const int r = threadIdx.x & (kFpRows - 1);
      if (r < rows) {
        const int q = q0 + r;
        const int ii = fo ? n - 1 - q : q;
        for (int c = threadIdx.x / kFpRows; c < W; c += blockDim.x / kFpRows) {
          const int p = plo + c;
          float v = 0.f;
          if (p >= 0 && p < n) v = u[(size_t)(fi ? n - 1 - p : p) * n + ii];
          tile[r * ldw + c] = v;
        }
      }
    }
    __syncthreads();
    const int wmax2 = W - 2;
    for (int r = 0; r < rows; ++r) {
      const float *trow = tile + r * ldw;
#pragma unroll
      for (int g = 0; g < kFpPerThread; ++g) {
        if (!act[g]) continue;
        int c = min(max(ps[g], -2), n) - plo;
        c = min(max(c, 0), wmax2);
        float u1 = trow[c];
        float u2 = trow[c + 1];
        const uint32_t e2 = e[g] + A[g];
        if (check_first) u1 = (e[g] < one) ? u1 : 0.f;
        u2 = (e2 < one) ? u2 : 0.f;
        P[g] += u1 + u2;
        Q[g] = fmaf((float)e[g], u1, Q[g]);
        Q[g] = fmaf((float)e2, u2, Q[g]);
        const uint32_t en = e[g] + B[g];
        const bool m = en >= A[g];
        e[g] = m ? en - A[g] : en;
        ps[g] -= m ? 1 : 0;
      }
    }
  }

  const float inv = 1.0f / (float)one;
#pragma unroll
  for (int g = 0; g < kFpPerThread; ++g) {
    if (!act[g]) continue;
    const float qprev = __shfl_up(Q[g], 1, 64);
    if (lane >= 1 && k <= grp.kmax && k < M) {
      sino[(size_t)lrow[g] * M + k] = fmaf(qprev - Q[g], inv, P[g]);
    }
  }
}

int launch_radon_fwd(const ct_plan *p, const float *u, float *out, hipStream_t s) {
  dim3 grid(p->n_groups, p->max_blk > 0 ? p->max_blk : 1);
  const int ldw = (p->wmax % 2 == 0) ? p->wmax + 1 : p->wmax;
  const size_t lds = sizeof(float) * kFpRows * ldw;
  hipLaunchKernelGGL(k_radon_fwd, grid, dim3(256), lds, s, u, p->g.n, p->g.n_bins, p->d_fp,
                     p->d_groups, p->d_regions, p->n_chunks, ldw, p->check_first ? 1 : 0, out);
  CT_TRY_HIP(hipGetLastError());
  return CT_OK;
}

}  // namespace ctpd
