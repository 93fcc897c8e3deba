// Internal declarations shared by the ctpd HIP sources (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/ctpd.h"

namespace ctpd {

// ---------------------------------------------------------------------------
// Error reporting: every ABI call returns a code and leaves a thread-local
// message.
void set_error(const std::string &msg);
void clear_error();

#define CT_TRY_HIP(expr)                                                        \
  do {                                                                          \
    hipError_t e_ = (expr);                                                     \
    if (e_ != hipSuccess) {                                                     \
      ::ctpd::set_error(std::string(#expr) + ": " + hipGetErrorString(e_));    \
      return CT_E_DEVICE;                                                       \
    }                                                                           \
  } while (0)

#define CT_TRY(expr)                                                            \
  do {                                                                          \
    int r_ = (expr);                                                            \
    if (r_ != CT_OK) return r_;                                                 \
  } while (0)

// Fixed-point bin coordinate: t * 2^30 as a 64-bit integer (§3.1 bin
// coordinate t = (x cos + y sin)/ds + (M-1)/2, quantized so that every
// kernel evaluates the same exact value for a pixel/angle pair).
constexpr int kFixBits = 30;
constexpr double kFixOne = 1073741824.0;  // 2^30

// Backprojection (R_h^*) per-angle constants: t(i, j) = t0 + i a + j b, each
// an exact multiple of 2^-30, so that the FP64 evaluation is exact.
struct BpAngle {
  double t0, a, b;
  double a32, b32;  // a 2^32 and b 2^32 (integers below 2^33, exact)
  int64_t b8_fix;   // 8 b 2^32 (exact: b is a multiple of 2^-30)
  int32_t l;       // sinogram row
  int32_t pad;
};

// Forward projection (R_h) per-angle constants in the walk frame: with the
// image re-indexed by (p, q) (transposed and/or mirrored), the fixed-point
// coordinate is T + p A + q B with A > 0 and 0 <= B <= A.
struct FpAngle {
  int64_t T;
  uint32_t A;
  uint32_t B;
  int32_t l;   // sinogram row
  int32_t pad;
  // the paired forward projector's position walk: pixels per bin 2^62 / A
  // and pixels moved per row B 2^32 / A, both in units of 2^-32, rounded
  uint64_t dfix;
  uint64_t dlt;
};

// Position walk of the paired forward projector.  For strip k (bin k) in
// walk row q, s = (k 2^30 - T - q B) / A is where the strip starts along the
// row: its pixels are floor(s + 1) ... (the boundary pixel of an integer s
// goes to the strip before, whose last pixel it is with weight 1 on bin k: the
// same contribution).  The walk keeps y = 2^32 (s + 1) as a 64-bit fixed-point
// number whose high word is the pixel index and low word the fraction g; the
// first pixel's interpolation weight is alpha = (1 - g) A 2^-30, and strip
// k + 1 starts where y + dfix floors.  y of one strip and row, rounded to
// 2^-32 in the same way on host and device (a correctly rounded division).
__host__ __device__ inline uint64_t walk_y0(int64_t k, int64_t q, int64_t T, uint32_t A,
                                            uint32_t B) {
  const int64_t num = k * ((int64_t)1 << kFixBits) - T - q * (int64_t)B;
  const double s = (double)num / (double)A + 1.0;
  return (uint64_t)(int64_t)rint(s * 4294967296.0);
}

// A group of up to kFpGroup angles of the same walk class, processed by one
// workgroup (one wave per kFpPerThread angles, 64 bins per workgroup).
constexpr int kFpWaves = 8;
constexpr int kFpThreads = 64 * kFpWaves;
constexpr int kFpPerThread = 2;
constexpr int kFpGroup = kFpWaves * kFpPerThread;  // 16 angles
constexpr int kFpStrips = 64;                       // strips per workgroup (63 outputs)
constexpr int kFpRows = 32;                         // image rows staged per chunk
constexpr int kFpMaxWidth = 192;                    // staged columns per chunk
constexpr int kFpPrefetch = kFpRows * kFpMaxWidth / kFpThreads;  // staged pixels per thread

// Paired variant: 2 angles whose walk constants (T, A, B) are identical
// share one walk.  A workgroup of kPrWaves waves owns kPrPairs pairs and a
// block of kPrStrips strips (kPrStrips - 1 output bins); a wave owns two
// pairs, its lanes in groups of 16 strips: lanes 0-15 pair A strips 0-15,
// 16-31 pair B strips 0-15, 32-47 pair A strips 16-31, 48-63 pair B strips
// 16-31.  So each half-wave reads 16 strips of two neighbouring angles at
// nearly the same staged positions: at most ~25 distinct columns, within the
// 32 LDS banks.
constexpr int kPrWaves = 4;
constexpr int kPrPairs = 2 * kPrWaves;
constexpr int kPrStrips = 32;
// Four angles per walk (theta, pi/2 - theta, pi - theta, pi/2 + theta): the
// same lane layout with quadruples in place of pairs, eight waves per
// workgroup sharing the four staged copies; used for images of at least
// kQuadMinN pixels a side.
constexpr int kQuadWaves = 8;
constexpr int kQuadItems = 2 * kQuadWaves;
constexpr int kQuadMinN = 1024;
constexpr int kMultiMaxWidth = 128;  // staged columns per chunk

// Strip offset and pair (0 = A, 1 = B) of lane `lane` of a paired wave.
__host__ __device__ inline int pr_strip(int lane) { return ((lane >> 5) << 4) | (lane & 15); }
__host__ __device__ inline int pr_pair(int lane) { return (lane >> 4) & 1; }

struct FpGroup {
  int32_t first;  // index into the FpAngle array (pairs: pair index, 2 entries each)
  int32_t count;  // angles (pairs) in the group (<= kFpGroup, kPrPairs)
  int32_t cls;    // bit0 transpose (walk columns), bit1 mirror inner, bit2 mirror outer
  int32_t kmin;   // first bin that can receive a nonzero value
  int32_t kmax;   // last such bin
  int32_t nblk;   // workgroups needed along the bins
  int32_t region; // offset of this group's (block, chunk) region table
  int32_t range;  // offset of this group's per-block active chunk ranges
  int32_t clss;   // multi-angle plans: class of angle s of each set in byte s
  int32_t pad;
};

// Backprojection tiling: 256 threads, 32 x 64 pixels, 8 pixels per thread
// (rows ty, ty + 8, ..., ty + 56).
constexpr int kBpTileI = 32;
constexpr int kBpTileJ = 64;
constexpr int kBpPix = 8;
constexpr int kBpRowStep = 8;
constexpr int kBpChunk = 16;    // angles staged per chunk
constexpr int kBpPrefetch = 8;  // staged pairs per thread: kBpChunk * seg <= 2048
// mirror pairs per staged chunk when a segment needs two rounds of 64 bins
// (8 when it fits one); the slice heuristics count chunks of this size
constexpr int kBpPairChunk = kBpChunk / 4;
constexpr int kBppPix = 4;                  // pixels per thread of the mirror-pair kernel
constexpr int kBppTileJ = kBpRowStep * kBppPix;  // its tiles: kBpTileI x kBppTileJ

// FFT plan (mixed radix 8/4/3/2, Stockham in LDS).
struct FftPlan {
  int32_t L;
  int32_t npass;
  int32_t radix[24];
  uint64_t code;  // radix of pass i in bits [4 i, 4 i + 4) (a scalar the kernels decode)
  // 1: radix-8 passes spread each butterfly over a quad of lanes (set where a
  // single problem's row block has fewer butterflies than a workgroup has
  // threads); fixed per length, so batches compute bitwise as single problems
  int32_t quad8;
};

}  // namespace ctpd

// Opaque ABI objects.
struct ct_plan {
  ct_geom g;
  int device;
  // backprojection
  ctpd::BpAngle *d_bp = nullptr;
  // mirror pairs (theta, pi - theta): entry 2c is angle l's geometry, entry
  // 2c + 1 its mirror image i -> n - 1 - i (row: the partner m, or -1)
  ctpd::BpAngle *d_bpp = nullptr;
  int n_bpp = 0;          // pairs (0: the one-angle backprojector)
  // backprojector of standalone calls and untuned solvers: 0 one angle at a
  // time, 4 or 8 mirror pairs with that many pixels per thread (a solver
  // keeps its own choice; the plan is never changed by a solver)
  int bp_kern0 = 4;
  uint64_t angles_hash = 0;  // FNV-1a of explicit angles (0: theta_l = pi l / N)
  std::vector<double> angles;  // the explicit angles (empty: theta_l = pi l / N)
  int walk_opt = 0;            // angles per walk the plan was created with (0: automatic)
  // set-up tunings done on this plan, (batch size, FFT pair next, fused
  // gradient-side update) -> choice, so that solvers created again for the
  // same batch size skip the timing (a memo only: each solver copies it)
  struct TuneEntry {
    int nb, fft, tvf, kern, S, tv_blocks, walk;
  };
  mutable std::vector<TuneEntry> tune_cache;
  int seg_pair = 0;       // staged bins per angle per tile of the pair kernel
  int seg = 0;  // staged bins per angle per tile
  int bp_slices = 1;           // angle slices of the backprojection grid
  float *d_bp_part = nullptr;  // [bp_slices][n][n] partial images (bp_slices > 1)
  // forward projection
  ctpd::FpAngle *d_fp = nullptr;
  ctpd::FpGroup *d_groups = nullptr;
  int2 *d_regions = nullptr;  // (p_lo, width) per (group, block, chunk)
  int2 *d_chunk_range = nullptr;  // first/last chunk per (group, block) meeting the image
  int2 *d_work = nullptr;         // (group, block) of every workgroup, in launch order
  int n_work = 0;
  int n_groups = 0;
  int max_blk = 0;
  int n_chunks = 0;
  int wmax = 0;     // widest staged region (columns)
  bool check_first = false;  // strips may hold no pixel of a row (|a| > 1)
  bool paired = false;       // angles share walks (slots > 1)
  int slots = 1;             // angles per walk: 1 or 2
  int chunk_rows = 16;       // image rows staged per chunk by the forward projector
  // scratch for standalone calls
  float *d_scratch_sino = nullptr;
  float *d_scratch_img = nullptr;
  double *d_red = nullptr;   // reduction partials
  int red_cap = 0;
};

struct ct_precond {
  int n;
  double sigma, tau, c, eps;
  float *d_mult = nullptr;   // [n/2+1][n] multiplier incl. 1/n^2
  float2 *d_tw = nullptr;    // twiddles exp(-2 pi i m / n)
  float2 *d_spec = nullptr;  // spectrum workspace [n/2+1][n]
  ctpd::FftPlan fp;
  // 1: the multiplier acts on the length-n^2 DFT of the column-major
  // vectorized image (circulant preconditioner), computed as the row pass,
  // a twiddle exp(-2 pi i j k1 / n^2), the column pass and their inverses
  int twist = 0;
};

namespace ctpd {

// ---- launchers (kernels live in the .hip files) ---------------------------
// out = c1 * R^*(v) + c2 * div_h(p)  (p may be null)
// nb problems of one geometry stored contiguously; part: nb * bp_slices
// partial images (NULL: the plan's own buffer, nb = 1 only).
// S: angle slices (0: the plan's choice).
// base (optional, nb images) is added to the result, base2 (optional)
// subtracted; out2 (optional, needs base) receives 2 out - base.
// The angle slices' sum and the epilogue of a sliced backprojection, not yet
// formed: out = base - base2 + c1 sum_s part[s] + c2 div_h(pfield).  A
// consumer that reads out once (the preconditioner's row pass) forms it on
// the fly instead of a separate combine pass.  S = 0: nothing deferred.
constexpr int kMaxDeferredSlices = 8;  // the plan's largest default slice count
constexpr int kMaxSlices = 16;         // the largest a solver's tuning tries
// slice counts whose sum the FFT row pass can form (else the combine pass)
inline bool deferrable_slices(int S) { return (S >= 2 && S <= kMaxDeferredSlices) || S == kMaxSlices; }
struct BpDeferred {
  const float *part = nullptr;  // [nb][S][n][n]
  int S = 0;
  const float *pfield = nullptr;
  float c1 = 0.f, c2 = 0.f, inv_h = 0.f;
  const float *base = nullptr, *base2 = nullptr;
};
// kern: the backprojector (0 one angle at a time, 4 or 8 mirror pairs with
// that many pixels per thread; < 0 the plan's default).
int launch_radon_adj(const ct_plan *p, const float *v, const float *pfield, float c1,
                     float c2, float *out, hipStream_t s, int nb = 1, float *part = nullptr,
                     int S = 0, int kern = -1, const float *base = nullptr,
                     const float *base2 = nullptr, float *out2 = nullptr,
                     BpDeferred *defer = nullptr);
// out = base + a x over count elements (nb problems contiguous).
int launch_axpy(int64_t count, const float *base, float a, const float *x, float *out,
                hipStream_t s);
// Objective terms of (C_h) in the problem's units, FP64: out[0] = 1/2 sum off
// D0 of (r - u0)^2, out[1] = max on D0 of (C - r)_+ (r = R_h u, raw), out[2] =
// sum |nabla_h u|.
int launch_objective(int N, int M, const float *r, const float *u0, const float *bound,
                     float bound_scalar, const uint32_t *mask, int n, float inv_h,
                     const float *u, double *partials, int cap, double *out, hipStream_t s);
// Optional epilogue of the forward projector: the PDRQS1 sinogram-side update
// applied to r = R(u)/beta per bin (see k_sino_update), instead of storing R(u).
struct SinoEpi {
  float inv_beta;
  float sigma;
  const float *target;
  const uint32_t *mask;
  float *vb1;
  float *s1;
  float *y1;
  float *r;
  int mode;      // 0 iterate, 1 caches only, 2 iterate and keep y1/r, 3 reverse sweep,
                 // 4 Algorithm CP dual step, 5 PDRQS2 residual, 6 ADMM z-step (mu in sigma),
                 // 7 PDRQ3 iterate, 8 PDRQ3 cache only
  float *q1 = nullptr;  // optional: the resolvent input 2 v1 - vb1 (modes 0, 2)
  int fit = 0;          // data term (modes 0, 2): CT_FIT_* of the C ABI
  const float *aux = nullptr;  // weights (weighted fit) or b on every bin (fit everywhere)
};
// out = R(u) (raw), or the epilogue when epi != nullptr
// Arguments of the gradient-side update (k_tv_update; the device code is in
// tv_update.hpp).  blocks > 0 in a forward launch: that many extra
// workgroups per problem run it next to the projection.
struct TvArgs {
  int n = 0;
  float inv_h = 0.f;
  const float *u = nullptr;
  float st = 0.f, radius = 0.f;
  float *vb2 = nullptr, *s2 = nullptr, *wout = nullptr;
  int mode = 0;
  float *q2out = nullptr, *ubar = nullptr;
  int blocks = 0;
};
// tv (optional): also run that update in the same launch when the paired
// kernel projects; *fused tells whether it did (else the caller launches it).
int launch_radon_fwd(const ct_plan *p, const float *u, float *out, hipStream_t s,
                     const SinoEpi *epi = nullptr, int nb = 1, const TvArgs *tv = nullptr,
                     bool *fused = nullptr);

// metal-trace estimate: dilation by a disk of radius <= kDilMaxRadius, R_h,
// D0 = {R_h chi > kappa}, bound = c0 u0 on D0 (when bound != nullptr)
constexpr int kDilMaxRadius = 16;
int launch_d0_estimate(const ct_plan *p, const float *u, float thr, int r, float kappa,
                       float *chi, float *proj, uint32_t *mask, const float *u0, float c0,
                       float *bound, hipStream_t s);

// ADMM's conjugate gradients: FP64 dot product into out[0]; u += a p,
// r -= a Hp with a = rz / pHp read on the device; p = z + (rz_new/rz_old) p
size_t dot_partials_needed();
int launch_dot(const float *x, const float *y, int64_t count, double *partials, double *out,
               hipStream_t s);
int launch_cg_update(int64_t count, const double *rz, const double *pHp, const float *p,
                     const float *Hp, float *u, float *r, hipStream_t s);
int launch_cg_dir(int64_t count, const double *rz_new, const double *rz_old, const float *z,
                  float *p, hipStream_t s);

int launch_grad(int n, float inv_h, const float *u, float *p, hipStream_t s);
int launch_div(int n, float inv_h, const float *p, float *d, hipStream_t s);
int launch_tv_project(int n, const float *q, float radius, float *w, hipStream_t s);
int launch_prox_sino(int N, int M, const float *q, float step, const float *u0,
                     const float *bound, const uint32_t *mask, float *y, hipStream_t s);

// Fused dual updates of PDRQS1.
// mode 0: full step; mode 1: cache only (s1 = vb1 + sigma r); mode 2: full step and
// write y1 and r for the gap record.
int launch_sino_update(int N, int M, const float *rraw, float inv_beta, float sigma,
                       const float *target, const uint32_t *mask, float *vb1, float *s1,
                       float *y1, float *rout, int mode, hipStream_t s);
// q2out (optional): the resolvent input 2 v2 - vb2 (modes 0, 2).  ubar
// (optional, modes 0, 2): bar u += max(2 u - bar u, 0) - u (u >= 0 variant).
int launch_tv_update(int n, float inv_h, const float *u, float sigtau, float radius,
                     float *vb2, float *s2, float *wout, int mode, hipStream_t s, int nb = 1,
                     float *q2out = nullptr, float *ubar = nullptr);
// Reverse sweep of unrolled PDRQS1 (see unrolled.hip).
int launch_sino_reverse(int N, int M, int nb, float sigma, const float *V1, const float *q1,
                        const float *target, const uint32_t *mask, float *P, float *Q1,
                        float *bbar, hipStream_t s);
int launch_tv_reverse(int n, int nb, float sigtau, float rho, const float *V2, const float *q2,
                      float *Q2, float *G, double *partials, double *acc, hipStream_t s);
int launch_img_tail(int n, int nb, float sigtau, float inv_h, const float *Utmp,
                    const float *Q2, const float *Utot, float *Uout, float *V2out,
                    hipStream_t s);
size_t tv_reverse_partials(int n, int nb);
int launch_build_target(int N, int M, const float *u0, const float *bound, float bscalar,
                        const uint32_t *mask, float inv_beta, float *target, hipStream_t s);

// FFT-based multiplier application: out = (base ? base : 0) + F^{-1}(mult F(y)).
// nb problems stored contiguously; spec: nb spectra (NULL: the
// preconditioner's own buffer, nb = 1 only).
// y == nullptr with ydef: y is the deferred backprojection ydef (S > 1)
int launch_apply_mult(const ct_precond *pc, const float *mult, const float *y,
                      const float *base, float *out, hipStream_t s, int nb = 1,
                      float2 *spec = nullptr, const BpDeferred *ydef = nullptr);

// Reductions (FP64, deterministic two-level).
int launch_norm2(const float *x, int64_t count, double *partials, int cap, double *out,
                 hipStream_t s);
int launch_scale_by_inv(const float *x, int64_t count, const double *norm, float *y,
                        hipStream_t s);
int launch_nonfinite(const float *x, int64_t count, int *flag, hipStream_t s);
// Gap terms: out[0] = 1/2 sum_off (r - b)^2, out[1] = sum_off (y1^2/2 + y1 b) + sum_on y1 C,
// out[2] = max_on (C - r)_+
int launch_sino_gap(int N, int M, const float *r, const float *y1, const float *target,
                    const uint32_t *mask, double *partials, int cap, double *out,
                    hipStream_t s);
// out[0] = sum |nabla u| (with 1/h), out[1] = sum (u - uprev)^2, out[2] = sum z^2
int launch_img_gap(int n, float inv_h, const float *u, const float *uprev, const float *z,
                   double *partials, int cap, double *out, hipStream_t s);

int reduction_partials_needed();

// FFT plan helpers
bool fft_factor(int L, FftPlan *fp);

}  // namespace ctpd
