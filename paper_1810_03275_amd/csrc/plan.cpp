// Projector plan: per-angle fixed-point tables and the forward projector's
// work list (thesis §3.1 geometry), built on the host in FP64/int64.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <tuple>
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

// Everything a plan holds, computed on the host.
struct HostPlan {
  std::vector<BpAngle> bp;
  std::vector<BpAngle> bpp;  // mirror pairs, two entries each (empty: unpaired)
  std::vector<FpAngle> dev;
  std::vector<FpGroup> groups;
  std::vector<int2> regions, ranges;
  std::vector<int2> work;  // (group, block) per forward workgroup, in launch order
  int seg = 0, seg_pair = 0, bp_slices = 1, n_groups = 0, max_blk = 0, n_chunks = 0, wmax = 0;
  bool check_first = false, paired = false;
  int slots = 1, chunk_rows = 16;
};

// Launch order of the forward workgroups.  Every (group, block) is one
// workgroup (a group without blocks still gets block 0, which writes its
// zero bins); its cost is the number of (wave, staged chunk) pairs it runs.
// The list is sorted by decreasing cost, so that the workgroups dispatched
// last, when the device drains, are the short ones.
static void schedule_work(HostPlan *p) {
  struct Item {
    int cost, g, b;
  };
  std::vector<Item> items;
  for (int gi = 0; gi < (int)p->groups.size(); ++gi) {
    const FpGroup &G = p->groups[gi];
    const int nb = G.nblk > 0 ? G.nblk : 1;
    for (int b = 0; b < nb; ++b) {
      int cost = 0;
      if (b < G.nblk) {
        const int2 r = p->ranges[G.range + b];
        cost = r.y >= r.x ? (r.y - r.x + 1) * G.count : 0;
      }
      items.push_back({cost, gi, b});
    }
  }
  std::stable_sort(items.begin(), items.end(),
                   [](const Item &x, const Item &y) { return x.cost > y.cost; });
  p->work.clear();
  for (const Item &it : items) p->work.push_back(make_int2(it.g, it.b));
}

static int plan_host(const ct_geom *g, const double *angles, const ct_plan_opts &opt,
                     HostPlan *p) {
  const int n = g->n, N = g->n_angles, M = g->n_bins;
  const double h = g->h, ds = g->ds;
  std::vector<BpAngle> &bp = p->bp;
  bp.assign(N, BpAngle{});
  std::vector<FpAngle> fp(N);
  std::vector<int> cls(N);
  bool check_first = false;
  // cos and sin of the default angles theta_l = pi l / N come from one
  // octant, so that angles related by pi/2 - theta or 3pi/2 - theta get
  // exactly swapped / negated values (their walks then coincide exactly).
  auto trig = [&](int l, double &c, double &s) {
    if (angles || N % 2 != 0) {
      const double th = angles ? angles[l] : M_PI * (double)l / (double)N;
      c = std::cos(th);
      s = std::sin(th);
      return;
    }
    if (4 * l <= N) {
      c = std::cos(M_PI * l / N);
      s = std::sin(M_PI * l / N);
    } else if (2 * l <= N) {
      const int m = N / 2 - l;
      c = std::sin(M_PI * m / N);
      s = std::cos(M_PI * m / N);
    } else if (4 * l < 3 * N) {
      const int m = l - N / 2;
      c = -std::sin(M_PI * m / N);
      s = std::cos(M_PI * m / N);
    } else {
      const int m = N - l;
      c = -std::cos(M_PI * m / N);
      s = std::sin(M_PI * m / N);
    }
  };
  for (int l = 0; l < N; ++l) {
    double c, s;
    trig(l, c, s);
    const double a = h * c / ds, b = h * s / ds;
    const int64_t A30 = std::llround(a * kFixOne);
    const int64_t B30 = std::llround(b * kFixOne);
    // walk frame: the inner coefficient is the larger one, both made >= 0
    // by mirroring; (p, q) = (0, 0) is image pixel (i0, j0)
    const bool tr = std::llabs(A30) < std::llabs(B30);
    const int64_t Ci = tr ? B30 : A30, Co = tr ? A30 : B30;
    const bool fi = Ci < 0, fo = Co < 0;
    const int i0 = tr ? (fo ? n - 1 : 0) : (fi ? n - 1 : 0);
    const int j0 = tr ? (fi ? n - 1 : 0) : (fo ? n - 1 : 0);
    const double x = h * (i0 - (n - 1) / 2.0), y = h * (j0 - (n - 1) / 2.0);
    const double t_origin = (x * c + y * s) / ds + (M - 1) / 2.0;
    const int64_t Tw = std::llround(t_origin * kFixOne);
    // image frame: t(i, j) = T30 + i A30 + j B30 (same integers as the walk)
    const int64_t T30 = Tw - (int64_t)i0 * A30 - (int64_t)j0 * B30;
    bp[l].t0 = (double)T30 / kFixOne;
    bp[l].a = (double)A30 / kFixOne;
    bp[l].b = (double)B30 / kFixOne;
    bp[l].a32 = (double)(A30 * 4);
    bp[l].b32 = (double)(B30 * 4);
    bp[l].b8_fix = B30 * 4 * 8;
    bp[l].l = l;
    bp[l].pad = 0;
    const int64_t Ai = fi ? -Ci : Ci, Bo = fo ? -Co : Co;
    if (Ai > (int64_t)1 << kFixBits) check_first = true;
    fp[l].T = Tw;
    fp[l].A = (uint32_t)Ai;
    fp[l].B = (uint32_t)Bo;
    fp[l].l = l;
    fp[l].pad = 0;
    {
      using u128 = unsigned __int128;
      const u128 a = (u128)(uint64_t)Ai;
      fp[l].dfix = (uint64_t)((((u128)1 << 62) + a / 2) / a);
      fp[l].dlt = (uint64_t)((((u128)(uint64_t)Bo << 32) + a / 2) / a);
    }
    cls[l] = (tr ? 1 : 0) | (fi ? 2 : 0) | (fo ? 4 : 0);
  }
  double max_extent = 0.0;  // largest detector span of a tile, in bins
  for (int l = 0; l < N; ++l)
    max_extent = std::max(max_extent, (kBpTileI - 1) * std::fabs(bp[l].a) +
                                          (kBpTileJ - 1) * std::fabs(bp[l].b));
  p->seg = (int)std::ceil(max_extent) + 2;
  {
    double ext = 0.0;
    for (int l = 0; l < N; ++l)
      ext = std::max(ext, (kBpTileI - 1) * std::fabs(bp[l].a) + (kBppTileJ - 1) * std::fabs(bp[l].b));
    p->seg_pair = (int)std::ceil(ext) + 2;
  }
  if (kBpChunk * p->seg > 256 * kBpPrefetch) {
    set_error("projector plan: backprojection segment too long (ds/h too small)");
    return CT_E_UNSUPPORTED;
  }
  // Mirror pairs for the backprojection: angle m with A30_m = -A30_l,
  // B30_m = B30_l and T30_m = T30_l + (n - 1) A30_l puts pixel (n - 1 - i, j)
  // exactly where l puts pixel (i, j) (for the default angles, l and N - l).
  // Angles without a partner are paired with their own mirror image and a
  // zero sinogram row.  Used when at least half of the angles pair up.
  {
    auto fix = [](double x) { return (int64_t)std::llround(x * kFixOne); };
    std::map<std::tuple<int64_t, int64_t, int64_t>, int> by_geom;
    for (int l = 0; l < N; ++l) by_geom.emplace(std::make_tuple(fix(bp[l].a), fix(bp[l].b), fix(bp[l].t0)), l);
    std::vector<char> used(N, 0);
    std::vector<BpAngle> pairs;
    int paired_angles = 0;
    for (int l = 0; l < N; ++l) {
      if (used[l]) continue;
      used[l] = 1;
      const int64_t A30 = fix(bp[l].a), B30 = fix(bp[l].b), T30 = fix(bp[l].t0);
      const int64_t Tm = T30 + (int64_t)(n - 1) * A30;
      int m = -1;
      const auto it = by_geom.find(std::make_tuple(-A30, B30, Tm));
      if (it != by_geom.end() && it->second != l && !used[it->second]) {
        m = it->second;
        used[m] = 1;
        paired_angles += 2;
      }
      BpAngle mir = bp[l];
      mir.t0 = (double)Tm / kFixOne;
      mir.a = (double)(-A30) / kFixOne;
      mir.a32 = (double)(-A30 * 4);
      mir.l = m;
      pairs.push_back(bp[l]);
      pairs.push_back(mir);
    }
    // the table is kept whenever the angles pair, so that a solver may choose
    // the pair kernel even when the plan's default is one angle at a time
    if (n >= 2 && 2 * paired_angles >= N) p->bpp = pairs;
    if ((opt.bp_kernel == CT_BP_PAIRS4 || opt.bp_kernel == CT_BP_PAIRS8) && p->bpp.empty()) {
      set_error("ct_plan_create: mirror-pair backprojection needs angles that pair as "
                "theta, pi - theta");
      return CT_E_UNSUPPORTED;
    }
  }
  {
    // workgroups: tiles (of the left half when paired) x angle slices
    const bool pairs = !p->bpp.empty() && opt.bp_kernel != CT_BP_ONE_ANGLE;
    const int ni = pairs ? (n + 1) / 2 : n;
    const int tj = pairs ? (opt.bp_kernel == CT_BP_PAIRS8 ? kBpTileJ : kBppTileJ) : kBpTileJ;
    const int tiles = ((ni + kBpTileI - 1) / kBpTileI) * ((n + tj - 1) / tj);
    const int items = pairs ? (int)(p->bpp.size() / 2) / kBpPairChunk : N / kBpChunk;
    int S = (1024 + tiles - 1) / tiles;
    S = std::min(S, kMaxDeferredSlices);
    S = std::min(S, std::max(1, items / 2));
    p->bp_slices = std::max(S, 1);
  }
  p->check_first = check_first;

  const int64_t one = (int64_t)1 << kFixBits;

  // Angles with identical walk constants can share one walk: for equispaced
  // angles theta, pi/2 - theta, pi - theta and pi/2 + theta.  Pairs are used
  // when at least half of the angles pair up, else one angle per walk.  An
  // angle without a partner is paired with a copy of itself whose results are
  // discarded (row l = -1).  A plan whose staged windows come out wider than
  // the paired kernel's limit (large ds/h) falls back to one angle per walk.
  std::vector<std::vector<int>> keysets;
  {
    std::map<std::tuple<int64_t, uint32_t, uint32_t>, std::vector<int>> by_key;
    for (int l = 0; l < N; ++l) by_key[std::make_tuple(fp[l].T, fp[l].A, fp[l].B)].push_back(l);
    for (auto &kv : by_key) keysets.push_back(kv.second);
  }
  auto complete = [&](int SL) {
    int c = 0;
    for (auto &v : keysets) c += (int)(v.size() / SL) * SL;
    return c;
  };
  std::vector<int> modes;
  {
    // automatic: four angles per walk for large images whose angles form
    // quadruples (there the projector is bound by VALU issue and the grid is
    // large enough for workgroups of 16 quadruples), else pairs, else one
    // (a forced mode whose windows come out too wide falls back to the next)
    const int forced = opt.fwd_angles_per_walk;
    const bool quads = N >= 4 && 2 * complete(4) >= N;
    const bool pairs = N >= 2 && 2 * complete(2) >= N;
    if (forced == 4 || (forced == 0 && n >= kQuadMinN && quads)) modes.push_back(4);
    if (forced == 2 || ((forced == 0 || forced == 4) && pairs)) modes.push_back(2);
    modes.push_back(1);
  }
  for (size_t attempt = 0; attempt < modes.size(); ++attempt) {
    const int SL = modes[attempt];
    const bool multi = SL > 1;
    const int rows_c = kFpRows;
    const int n_chunks = (n + rows_c - 1) / rows_c;
    const int max_width = multi ? kMultiMaxWidth : kFpMaxWidth;
    const int per_group = (SL == 4) ? kQuadItems : (SL == 2) ? kPrPairs : kFpGroup;
    const int strips = multi ? kPrStrips : kFpStrips;  // strips per block (one halo strip)

    // Work items (angles, or sets of SL angles) in class order; rep[i] holds
    // the walk constants of item i, icls[i] its classes (one per slot).
    std::vector<FpAngle> rep;
    std::vector<FpAngle> &dev = p->dev;  // the device table (SL entries per item)
    dev.clear();
    std::vector<std::vector<int>> icls;
    if (multi) {
      std::vector<std::vector<int>> items;  // angles, -1 - l for a discarded copy of l
      for (auto &v : keysets)
        for (size_t i = 0; i < v.size(); i += SL) {
          std::vector<int> it;
          for (int s = 0; s < SL && i + s < v.size(); ++s) it.push_back(v[i + s]);
          const size_t real = it.size();
          for (size_t s = 0; it.size() < (size_t)SL; ++s) it.push_back(-1 - it[s % real]);
          // order the slots by class so that items of one group align
          std::stable_sort(it.begin(), it.end(), [&](int x, int y) {
            const int lx = x >= 0 ? x : -1 - x, ly = y >= 0 ? y : -1 - y;
            return cls[lx] < cls[ly];
          });
          items.push_back(it);
        }
      auto key = [&](const std::vector<int> &it) {
        std::vector<int> kc;
        for (int x : it) kc.push_back(cls[x >= 0 ? x : -1 - x]);
        return kc;
      };
      std::stable_sort(items.begin(), items.end(),
                       [&](const std::vector<int> &x, const std::vector<int> &y) {
                         const auto kx = key(x), ky = key(y);
                         if (kx != ky) return kx < ky;
                         return x[0] < y[0];
                       });
      for (auto &it : items) {
        const int l0 = it[0] >= 0 ? it[0] : -1 - it[0];
        rep.push_back(fp[l0]);
        for (int x : it) {
          FpAngle f = fp[x >= 0 ? x : -1 - x];
          if (x < 0) f.l = -1;
          dev.push_back(f);
        }
        icls.push_back(key(it));
      }
    } else {
      std::vector<int> order(N);
      std::iota(order.begin(), order.end(), 0);
      std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return cls[x] < cls[y]; });
      for (int i = 0; i < N; ++i) {
        rep.push_back(fp[order[i]]);
        icls.push_back({cls[order[i]]});
      }
      dev = rep;
    }
    const int n_items = (int)rep.size();

    // Bins a group can reach and the staged column range of every
    // (block, chunk); returns the widest range.  The multi-angle kernels do
    // not clamp strip positions, so their ranges cover every position a lane
    // reaches; the one-angle kernel clamps positions to [-2, n].
    auto layout = [&](FpGroup &G, std::vector<int2> *out, std::vector<int2> *ranges) -> int {
      int64_t tmin = INT64_MAX, tmax = INT64_MIN;
      for (int a = 0; a < G.count; ++a) {
        const FpAngle &f = rep[G.first + a];
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
        G.nblk = (int)((kmax - kmin + 1 + (strips - 2)) / (strips - 1));
      }
      int wmax_g = 0;
      for (int b = 0; b < G.nblk; ++b) {
        const int64_t kb = G.kmin + (int64_t)b * (strips - 1);
        const int64_t klo = kb - 1, khi = kb + strips - 2;
        // Chunks where some strip of the block meets the image: strip k meets
        // row q iff ps(k+1, q) > 0 and ps(k, q) < n, and ps decreases along q,
        // so a chunk [q0, q1] can be skipped when ps(khi+1, q0) <= 0 or
        // ps(klo, q1) >= n for every angle of the group.
        int cf = n_chunks, cl = -1;
        for (int ch = 0; ch < n_chunks; ++ch) {
          const int64_t q0 = (int64_t)ch * rows_c;
          const int64_t q1 = std::min<int64_t>(q0 + rows_c, n) - 1;
          bool meets = false;
          for (int a = 0; a < G.count && !meets; ++a) {
            const FpAngle &f = rep[G.first + a];
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
          const int64_t q0 = (int64_t)ch * rows_c;
          const int64_t q1 = std::min<int64_t>(q0 + rows_c, n) - 1;
          int64_t lo = INT64_MAX, hi = INT64_MIN;
          for (int a = 0; a < G.count; ++a) {
            const FpAngle &f = rep[G.first + a];
            const int64_t ps_lo = ceil_div(klo * one - f.T - q1 * (int64_t)f.B, f.A);
            const int64_t ps_hi = ceil_div(khi * one - f.T - q0 * (int64_t)f.B, f.A);
            lo = std::min(lo, multi ? ps_lo : clamp64(ps_lo, -2, n));
            hi = std::max(hi, (multi ? ps_hi : clamp64(ps_hi, -2, n)) + 1);
          }
          lo -= 1;
          hi += 1;
          const int64_t W = hi - lo + 1;
          const bool active = ch >= cf && ch <= cl;
          // inactive chunks are never staged; keep their entry small
          if (out) out->push_back(active ? make_int2((int)lo, (int)W) : make_int2(0, 4));
          if (active) wmax_g = (int)std::max<int64_t>(wmax_g, W);
        }
      }
      return wmax_g;
    };

    std::vector<FpGroup> &groups = p->groups;
    std::vector<int2> &regions = p->regions, &ranges = p->ranges;
    groups.clear();
    regions.clear();
    ranges.clear();
    int wmax = 4, max_blk = 1;
    for (int i = 0; i < n_items;) {
      int j = i;
      while (j < n_items && j - i < per_group && icls[j] == icls[i]) ++j;
      FpGroup G{};
      G.first = i;
      G.cls = icls[i][0];
      G.clss = 0;
      for (size_t s = 0; s < icls[i].size() && s < 4; ++s) G.clss |= icls[i][s] << (8 * s);
      G.count = j - i;
      // fewer items per group when their strips spread too far apart
      while (G.count > 1 && layout(G, nullptr, nullptr) > max_width) G.count = (G.count + 1) / 2;
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
    p->paired = multi;
    p->slots = SL;
    p->chunk_rows = rows_c;
    if (wmax <= max_width) break;
    if (!multi) {
      set_error("projector plan: staged region wider than " + std::to_string(max_width) +
                " columns (too few angles for the group size)");
      return CT_E_UNSUPPORTED;
    }
  }
  if (p->regions.empty()) p->regions.push_back(make_int2(0, 4));
  if (p->ranges.empty()) p->ranges.push_back(make_int2(0, -1));
  schedule_work(p);
  return CT_OK;
}

// The forward projector's tables of a host plan, to the device.
static int upload_fwd(const HostPlan &hp, ct_plan *p) {
  p->check_first = hp.check_first;
  p->paired = hp.paired;
  p->slots = hp.slots;
  p->chunk_rows = hp.chunk_rows;
  p->n_groups = hp.n_groups;
  p->max_blk = hp.max_blk;
  p->n_chunks = hp.n_chunks;
  p->wmax = hp.wmax;
  p->n_work = (int)hp.work.size();
  CT_TRY_HIP(hipMalloc(&p->d_fp, sizeof(FpAngle) * hp.dev.size()));
  CT_TRY_HIP(hipMalloc(&p->d_groups, sizeof(FpGroup) * hp.groups.size()));
  CT_TRY_HIP(hipMalloc(&p->d_regions, sizeof(int2) * hp.regions.size()));
  CT_TRY_HIP(hipMalloc(&p->d_chunk_range, sizeof(int2) * hp.ranges.size()));
  CT_TRY_HIP(hipMalloc(&p->d_work, sizeof(int2) * hp.work.size()));
  CT_TRY_HIP(hipMemcpy(p->d_work, hp.work.data(), sizeof(int2) * hp.work.size(),
                       hipMemcpyHostToDevice));
  CT_TRY_HIP(hipMemcpy(p->d_chunk_range, hp.ranges.data(), sizeof(int2) * hp.ranges.size(),
                       hipMemcpyHostToDevice));
  CT_TRY_HIP(hipMemcpy(p->d_fp, hp.dev.data(), sizeof(FpAngle) * hp.dev.size(),
                       hipMemcpyHostToDevice));
  CT_TRY_HIP(hipMemcpy(p->d_groups, hp.groups.data(), sizeof(FpGroup) * hp.groups.size(),
                       hipMemcpyHostToDevice));
  CT_TRY_HIP(hipMemcpy(p->d_regions, hp.regions.data(), sizeof(int2) * hp.regions.size(),
                       hipMemcpyHostToDevice));
  return CT_OK;
}

int build_plan(const ct_geom *g, const double *angles, const ct_plan_opts &opt, ct_plan *p) {
  HostPlan hp;
  CT_TRY(plan_host(g, angles, opt, &hp));
  const int n = g->n, N = g->n_angles;
  p->seg = hp.seg;
  p->seg_pair = hp.seg_pair;
  if (hp.bpp.empty() || opt.bp_kernel == CT_BP_ONE_ANGLE)
    p->bp_kern0 = 0;
  else
    p->bp_kern0 = opt.bp_kernel == CT_BP_PAIRS8 ? 8 : 4;
  p->angles_hash = 0;
  p->angles.clear();
  if (angles) {
    p->angles.assign(angles, angles + N);
    // FNV-1a over the angles' bytes: part of the tuning cache's key
    uint64_t hsh = 1469598103934665603ull;
    const unsigned char *b = reinterpret_cast<const unsigned char *>(angles);
    for (size_t q = 0; q < sizeof(double) * (size_t)N; ++q) {
      hsh ^= b[q];
      hsh *= 1099511628211ull;
    }
    p->angles_hash = hsh ? hsh : 1;
  }
  p->walk_opt = opt.fwd_angles_per_walk;
  p->bp_slices = hp.bp_slices;
  CT_TRY_HIP(hipMalloc(&p->d_bp, sizeof(BpAngle) * N));
  p->n_bpp = (int)(hp.bpp.size() / 2);
  if (p->n_bpp > 0) {
    CT_TRY_HIP(hipMalloc(&p->d_bpp, sizeof(BpAngle) * hp.bpp.size()));
    CT_TRY_HIP(hipMemcpy(p->d_bpp, hp.bpp.data(), sizeof(BpAngle) * hp.bpp.size(),
                         hipMemcpyHostToDevice));
  }
  if (p->bp_slices > 1)
    CT_TRY_HIP(hipMalloc(&p->d_bp_part, sizeof(float) * (size_t)p->bp_slices * n * n));
  CT_TRY_HIP(hipMemcpy(p->d_bp, hp.bp.data(), sizeof(BpAngle) * N, hipMemcpyHostToDevice));
  return upload_fwd(hp, p);
}

// A plan holding only the geometry and the forward projector's tables for
// `walk` angles per walk (1, 2 or 4, falling back as plan creation does when
// the staged windows come out too wide), built from the angles of `base`.
// Only launch_radon_fwd may be given it.
int build_fwd_plan(const ct_plan *base, int walk, ct_plan *p) {
  ct_plan_opts opt{CT_BP_AUTO, walk};
  HostPlan hp;
  CT_TRY(plan_host(&base->g, base->angles.empty() ? nullptr : base->angles.data(), opt, &hp));
  p->g = base->g;
  p->device = base->device;
  p->angles_hash = base->angles_hash;
  p->walk_opt = walk;
  p->n_bpp = 0;
  p->bp_slices = 1;
  return upload_fwd(hp, p);
}

// Host replay of the forward projector's walk over every (group, block, wave,
// lane, staged row) of a plan: each LDS read must fall inside the staged
// window of its chunk, and every row that the kernel skips must hold no pixel
// of any strip of the block.  The same integer arithmetic as on the device:
// the exact walk of the one-angle kernel, the fixed-point walk of the paired
// one.
int check_plan(const ct_geom *g, const double *angles, const ct_plan_opts &opt,
               int64_t *steps) {
  HostPlan hp;
  CT_TRY(plan_host(g, angles, opt, &hp));
  const int n = g->n;
  const int64_t one = (int64_t)1 << kFixBits;
  int64_t count = 0;
  {
    // the launch list holds every (group, block) exactly once
    std::vector<int> base(hp.groups.size() + 1, 0);
    for (size_t gi = 0; gi < hp.groups.size(); ++gi)
      base[gi + 1] = base[gi] + std::max(hp.groups[gi].nblk, 1);
    std::vector<char> seen(base.back(), 0);
    bool ok = hp.work.size() == seen.size();
    for (const int2 &w : hp.work) {
      if (!ok) break;
      ok = w.x >= 0 && w.x < (int)hp.groups.size() && w.y >= 0 &&
           w.y < std::max(hp.groups[w.x].nblk, 1) && !seen[base[w.x] + w.y];
      if (ok) seen[base[w.x] + w.y] = 1;
    }
    if (!ok) {
      set_error("plan check: the forward launch list is not a permutation of the workgroups");
      return CT_E_INVALID;
    }
  }
  for (const FpGroup &G : hp.groups) {
    const int slots = G.count;
    for (int b = 0; b < G.nblk; ++b) {
      const int2 cr = hp.ranges[G.range + b];
      const int2 *reg = hp.regions.data() + G.region + (size_t)b * hp.n_chunks;
      for (int w = 0; w < slots; ++w) {
        const FpAngle fa = hp.dev[(size_t)hp.slots * (G.first + w)];
        const int strips = hp.paired ? kPrStrips : kFpStrips;
        for (int lane = 0; lane < strips; ++lane) {
          const int64_t k = G.kmin + (int64_t)b * (strips - 1) - 1 + lane;
          // rows of skipped chunks: no pixel of the strip inside the image
          for (int64_t q = 0; q < n; ++q) {
            const int64_t ch = q / hp.chunk_rows;
            if (ch >= cr.x && ch <= cr.y) continue;
            const int64_t ps = ceil_div(k * one - fa.T - q * (int64_t)fa.B, fa.A);
            const int64_t pe = ceil_div((k + 1) * one - fa.T - q * (int64_t)fa.B, fa.A);
            if (pe > ps && ps < n && pe > 0) {
              set_error("plan check: a skipped row holds pixels of strip " + std::to_string(k));
              return CT_E_INVALID;
            }
          }
          if (cr.x > cr.y) continue;
          const int64_t q_first = (int64_t)cr.x * hp.chunk_rows;
          if (hp.paired) {
            // the paired kernel's fixed-point walk (walk_y0 + lane dfix, then
            // dlt per row): the first pixel is read when it lies in the
            // strip, the second one when the strip holds two pixels
            uint64_t y = walk_y0(k - lane, q_first, fa.T, fa.A, fa.B) + (uint64_t)lane * fa.dfix;
            const bool two = (fa.dfix >> 32) != 0;
            const uint32_t dlo = (uint32_t)fa.dfix;
            if (!two && !hp.check_first) {
              set_error("plan check: a strip narrower than a pixel in a kernel that reads "
                        "every first pixel");
              return CT_E_INVALID;
            }
            for (int ch = cr.x; ch <= cr.y; ++ch) {
              const int rows = std::min(hp.chunk_rows, n - ch * hp.chunk_rows);
              const int2 rg = reg[ch];
              if (rg.y > hp.wmax) {
                set_error("plan check: window wider than the plan's width");
                return CT_E_INVALID;
              }
              for (int r = 0; r < rows; ++r) {
                const int64_t X = (int64_t)(int32_t)(uint32_t)(y >> 32);
                const uint32_t lo = (uint32_t)y;
                const bool in1 = two || lo >= 0u - dlo;
                const bool in2 = two && lo > ~dlo;
                const int64_t c = X - rg.x;
                const int64_t last = c + (in2 ? 1 : 0);
                if ((in1 || in2) && (c < 0 || last > rg.y - 1)) {
                  set_error("plan check: staged window misses strip " + std::to_string(k) +
                            " at row " + std::to_string(ch * hp.chunk_rows + r));
                  return CT_E_INVALID;
                }
                ++count;
                y -= fa.dlt;
              }
            }
            continue;
          }
          const int64_t num = k * one - fa.T - q_first * (int64_t)fa.B;
          int64_t pp = (int64_t)std::ceil((double)num / (double)fa.A);
          int64_t ee = pp * (int64_t)fa.A - num;
          if (ee < 0) {
            pp += 1;
            ee += fa.A;
          } else if (ee >= (int64_t)fa.A) {
            pp -= 1;
            ee -= fa.A;
          }
          if (ee < 0 || ee >= (int64_t)fa.A ||
              pp != ceil_div(num, fa.A)) {
            set_error("plan check: initial walk state is not exact");
            return CT_E_INVALID;
          }
          pp = clamp64(pp, -(1 << 29), 1 << 29);
          int64_t ps = pp;
          uint32_t e = (uint32_t)ee;
          for (int ch = cr.x; ch <= cr.y; ++ch) {
            const int rows = std::min(hp.chunk_rows, n - ch * hp.chunk_rows);
            const int2 rg = reg[ch];
            if (rg.y > hp.wmax) {
              set_error("plan check: window wider than the plan's width");
              return CT_E_INVALID;
            }
            for (int r = 0; r < rows; ++r) {
              const int64_t pos = clamp64(ps, -2, n);
              const int64_t c = pos - rg.x;
              if (c < 0 || c + 1 > rg.y - 1) {
                set_error("plan check: staged window misses strip " + std::to_string(k) +
                          " at row " + std::to_string(ch * hp.chunk_rows + r));
                return CT_E_INVALID;
              }
              ++count;
              const uint32_t en = e + fa.B;
              const bool below = en < fa.A;
              e = below ? en : en - fa.A;
              ps = ps - 1 + (below ? 1 : 0);
            }
          }
        }
      }
    }
  }
  if (steps) *steps = count;
  return CT_OK;
}

void free_plan(ct_plan *p) {
  if (!p) return;
  (void)hipFree(p->d_bp);
  (void)hipFree(p->d_bpp);
  (void)hipFree(p->d_bp_part);
  (void)hipFree(p->d_fp);
  (void)hipFree(p->d_groups);
  (void)hipFree(p->d_regions);
  (void)hipFree(p->d_chunk_range);
  (void)hipFree(p->d_work);
  (void)hipFree(p->d_scratch_sino);
  (void)hipFree(p->d_scratch_img);
  (void)hipFree(p->d_red);
}

}  // namespace ctpd
