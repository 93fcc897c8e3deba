// Projector plan: per-angle fixed-point tables and the forward projector's
// work list (thesis §3.1 geometry), built on the host in FP64/int64.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <string>

#include "common.hpp"

namespace ctpd {

namespace {

int64_t floor_div(int64_t a, int64_t b) {  // b > 0
  int64_t q = a / b;
  if ((a % b != 0) && (a < 0)) --q;
  return q;
}

int64_t ceil_div(int64_t a, int64_t b) {  // b > 0
  return -floor_div(-a, b);
}

int64_t clamp64(int64_t v, int64_t lo, int64_t hi) { return v < lo ? lo : (v > hi ? hi : v); }

}  // namespace

int build_plan(const ct_geom *g, const double *angles, ct_plan *p) {
  const int n = g->n, N = g->n_angles, M = g->n_bins;
  const double h = g->h, ds = g->ds;
  std::vector<BpAngle> bp(N);
  std::vector<FpAngle> fp(N);
  std::vector<int> cls(N);
  double max_span = 0.0;
  bool check_first = false;
  const double x0 = -h * (n - 1) / 2.0;
  for (int l = 0; l < N; ++l) {
    const double th = angles ? angles[l] : M_PI * (double)l / (double)N;
    const double c = std::cos(th), s = std::sin(th);
    const double a = h * c / ds, b = h * s / ds;
    const double t00 = (x0 * c + x0 * s) / ds + (M - 1) / 2.0;
    const int64_t A30 = std::llround(a * kFixOne);
    const int64_t B30 = std::llround(b * kFixOne);
    const int64_t T30 = std::llround(t00 * kFixOne);
    bp[l].t0 = (double)T30 / kFixOne;
    bp[l].a = (double)A30 / kFixOne;
    bp[l].b = (double)B30 / kFixOne;
    bp[l].b8_fix = B30 * 4 * 8;
    bp[l].l = l;
    bp[l].pad = 0;
    max_span = std::max(max_span, std::fabs(bp[l].a) + std::fabs(bp[l].b));
    // walk frame
    const bool tr = std::llabs(A30) < std::llabs(B30);
    int64_t Ci = tr ? B30 : A30, Co = tr ? A30 : B30, T = T30;
    bool fi = false, fo = false;
    if (Ci < 0) { T += (int64_t)(n - 1) * Ci; Ci = -Ci; fi = true; }
    if (Co < 0) { T += (int64_t)(n - 1) * Co; Co = -Co; fo = true; }
    if (Ci > (int64_t)1 << kFixBits) check_first = true;
    fp[l].T = T;
    fp[l].A = (uint32_t)Ci;
    fp[l].B = (uint32_t)Co;
    fp[l].l = l;
    fp[l].pad = 0;
    cls[l] = (tr ? 1 : 0) | (fi ? 2 : 0) | (fo ? 4 : 0);
  }
  double max_extent = 0.0;  // largest detector span of a tile, in bins
  for (int l = 0; l < N; ++l)
    max_extent = std::max(max_extent, (kBpTileI - 1) * std::fabs(bp[l].a) +
                                          (kBpTileJ - 1) * std::fabs(bp[l].b));
  p->seg = (int)std::ceil(max_extent) + 2;
  if (kBpChunk * p->seg > 256 * kBpPrefetch) {
    set_error("projector plan: backprojection segment too long (ds/h too small)");
    return CT_E_UNSUPPORTED;
  }
  {
    const int tiles = ((n + kBpTileI - 1) / kBpTileI) * ((n + kBpTileJ - 1) / kBpTileJ);
    int S = (1024 + tiles - 1) / tiles;
    S = std::min(S, 8);
    S = std::min(S, std::max(1, N / (2 * kBpChunk)));
    p->bp_slices = std::max(S, 1);
  }
  p->check_first = check_first;

  // group angles by class, kFpGroup at a time (angle order kept within a class)
  std::vector<int> order(N);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return cls[x] < cls[y]; });
  std::vector<FpAngle> fps(N);
  for (int i = 0; i < N; ++i) fps[i] = fp[order[i]];
  const int n_chunks = (n + kFpRows - 1) / kFpRows;
  const int64_t one = (int64_t)1 << kFixBits;

  // Bins a group can reach and the staged column range of every
  // (block, chunk); returns the widest range.
  auto layout = [&](FpGroup &G, std::vector<int2> *out, std::vector<int2> *ranges) -> int {
    int64_t tmin = INT64_MAX, tmax = INT64_MIN;
    for (int a = 0; a < G.count; ++a) {
      const FpAngle &f = fps[G.first + a];
      tmin = std::min(tmin, f.T);
      tmax = std::max(tmax, f.T + (int64_t)(n - 1) * ((int64_t)f.A + (int64_t)f.B));
    }
    int64_t kmin = floor_div(tmin, one);
    int64_t kmax = floor_div(tmax, one) + 1;
    kmin = std::max<int64_t>(kmin, 0);
    kmax = std::min<int64_t>(kmax, M - 1);
    if (kmin > kmax) {
      G.kmin = M;
      G.kmax = M - 1;
      G.nblk = 0;
    } else {
      G.kmin = (int)kmin;
      G.kmax = (int)kmax;
      G.nblk = (int)((kmax - kmin + 1 + (kFpStrips - 2)) / (kFpStrips - 1));
    }
    int wmax_g = 0;
    for (int b = 0; b < G.nblk; ++b) {
      const int64_t kb = G.kmin + (int64_t)b * (kFpStrips - 1);
      const int64_t klo = kb - 1, khi = kb + kFpStrips - 2;
      // Chunks where some strip of the block meets the image: strip k meets row
      // q iff ps(k+1, q) > 0 and ps(k, q) < n, and ps decreases along q, so a
      // chunk [q0, q1] can be skipped when ps(khi+1, q0) <= 0 or ps(klo, q1) >= n
      // for every angle of the group.
      int cf = n_chunks, cl = -1;
      for (int ch = 0; ch < n_chunks; ++ch) {
        const int64_t q0 = (int64_t)ch * kFpRows;
        const int64_t q1 = std::min<int64_t>(q0 + kFpRows, n) - 1;
        bool meets = false;
        for (int a = 0; a < G.count && !meets; ++a) {
          const FpAngle &f = fps[G.first + a];
          const int64_t right = ceil_div((khi + 1) * one - f.T - q0 * (int64_t)f.B, f.A);
          const int64_t left = ceil_div(klo * one - f.T - q1 * (int64_t)f.B, f.A);
          meets = right > 0 && left < n;
        }
        if (meets) {
          cf = std::min(cf, ch);
          cl = std::max(cl, ch);
        }
      }
      if (ranges) ranges->push_back(make_int2(cf, cl));
      for (int ch = 0; ch < n_chunks; ++ch) {
        const int64_t q0 = (int64_t)ch * kFpRows;
        const int64_t q1 = std::min<int64_t>(q0 + kFpRows, n) - 1;
        int64_t lo = INT64_MAX, hi = INT64_MIN;
        for (int a = 0; a < G.count; ++a) {
          const FpAngle &f = fps[G.first + a];
          const int64_t ps_lo = ceil_div(klo * one - f.T - q1 * (int64_t)f.B, f.A);
          const int64_t ps_hi = ceil_div(khi * one - f.T - q0 * (int64_t)f.B, f.A);
          lo = std::min(lo, clamp64(ps_lo, -2, n));
          hi = std::max(hi, clamp64(ps_hi, -2, n) + 1);
        }
        lo -= 1;
        hi += 1;
        const int W = (int)(hi - lo + 1);
        if (out) out->push_back(make_int2((int)lo, W));
        wmax_g = std::max(wmax_g, W);
      }
    }
    return wmax_g;
  };

  std::vector<FpGroup> groups;
  std::vector<int2> regions, ranges;
  int wmax = 4, max_blk = 1;
  for (int i = 0; i < N;) {
    int j = i;
    while (j < N && j - i < kFpGroup && cls[order[j]] == cls[order[i]]) ++j;
    FpGroup G{};
    G.first = i;
    G.cls = cls[order[i]];
    G.count = j - i;
    // fewer angles per group when their strips spread too far apart
    while (G.count > 1 && layout(G, nullptr, nullptr) > kFpMaxWidth) G.count = (G.count + 1) / 2;
    G.region = (int)regions.size();
    G.range = (int)ranges.size();
    const int w = layout(G, &regions, &ranges);
    wmax = std::max(wmax, w);
    max_blk = std::max(max_blk, G.nblk);
    groups.push_back(G);
    i += G.count;
  }
  p->n_groups = (int)groups.size();
  p->max_blk = max_blk;
  p->n_chunks = n_chunks;
  p->wmax = wmax;
  if (wmax > kFpMaxWidth) {
    set_error("projector plan: staged region wider than " + std::to_string(kFpMaxWidth) +
              " columns (too few angles for the group size)");
    return CT_E_UNSUPPORTED;
  }
  if (regions.empty()) regions.push_back(make_int2(0, 4));
  if (ranges.empty()) ranges.push_back(make_int2(0, -1));
  CT_TRY_HIP(hipMalloc(&p->d_bp, sizeof(BpAngle) * N));
  if (p->bp_slices > 1)
    CT_TRY_HIP(hipMalloc(&p->d_bp_part, sizeof(float) * (size_t)p->bp_slices * n * n));
  CT_TRY_HIP(hipMalloc(&p->d_fp, sizeof(FpAngle) * N));
  CT_TRY_HIP(hipMalloc(&p->d_groups, sizeof(FpGroup) * groups.size()));
  CT_TRY_HIP(hipMalloc(&p->d_regions, sizeof(int2) * regions.size()));
  CT_TRY_HIP(hipMalloc(&p->d_chunk_range, sizeof(int2) * ranges.size()));
  CT_TRY_HIP(hipMemcpy(p->d_chunk_range, ranges.data(), sizeof(int2) * ranges.size(),
                       hipMemcpyHostToDevice));
  CT_TRY_HIP(hipMemcpy(p->d_bp, bp.data(), sizeof(BpAngle) * N, hipMemcpyHostToDevice));
  CT_TRY_HIP(hipMemcpy(p->d_fp, fps.data(), sizeof(FpAngle) * N, hipMemcpyHostToDevice));
  CT_TRY_HIP(hipMemcpy(p->d_groups, groups.data(), sizeof(FpGroup) * groups.size(),
                       hipMemcpyHostToDevice));
  CT_TRY_HIP(hipMemcpy(p->d_regions, regions.data(), sizeof(int2) * regions.size(),
                       hipMemcpyHostToDevice));
  return CT_OK;
}

void free_plan(ct_plan *p) {
  if (!p) return;
  (void)hipFree(p->d_bp);
  (void)hipFree(p->d_bp_part);
  (void)hipFree(p->d_fp);
  (void)hipFree(p->d_groups);
  (void)hipFree(p->d_regions);
  (void)hipFree(p->d_chunk_range);
  (void)hipFree(p->d_scratch_sino);
  (void)hipFree(p->d_scratch_img);
  (void)hipFree(p->d_red);
}

}  // namespace ctpd
