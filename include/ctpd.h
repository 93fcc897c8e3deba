/*
 * ctpd: preconditioned primal-dual TV/metal CT reconstruction on AMD Instinct
 * MI355X (gfx950).  C ABI.
 *
 * Method: C. Schiffer, "TV-regularized CT reconstruction and metal artifact
 * reduction using inequality constraints with preconditioning" (2018,
 * arXiv:1810.03275).  Problem (C_h) of §3.2:
 *
 *   min_u  1/2 ||R_h u - u0||^2 on D\D0  +  lambda ||nabla_h u||_1
 *          subject to (R_h u)(l,k) >= C(l,k) for (l,k) in the metal trace D0,
 *
 * solved by Algorithm PDRQS1 (§4.4) with the inverse-norm + periodic-Laplacian
 * Fourier preconditioner (§4.3.1) on the normalized operator A = R_h/beta (§5.1).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Images are float32 [n][n], row-major, u[j][i] with j the y index and i the
 *   x index (§3.1 grid: pixel centres x_i = h (i - (n-1)/2), same for y_j).
 * - Sinograms are float32 [N][M], one contiguous row of M bins per angle.
 *   Bin k (0-based) has centre s_k = ds (k - (M-1)/2) (§3.1 detector).
 * - Gradient fields are float32 planar [2][n][n]: plane 0 the x difference,
 *   plane 1 the y difference (§3.1 nabla_h).
 * - Metal-trace masks are uint32 bitmasks [N][ceil(M/32)], bit (k & 31) of word
 *   k >> 5 set when bin k of angle l is in D0.
 * - Every array pointer is a DEVICE pointer owned by the caller (contiguous).
 *   The library never frees caller memory.  Opaque objects (plans,
 *   preconditioners, solvers) are created and destroyed by explicit calls and
 *   own their internal device memory.
 * - Work is enqueued on the given stream (a hipStream_t; NULL is the default
 *   stream).  Only calls that return host scalars synchronize that stream.
 * - Return value: CT_OK (0) or a negative CT_E_* code; ct_last_error() gives a
 *   message for the calling thread.  No exception crosses the ABI.
 */
#ifndef CTPD_H
#define CTPD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef void *ct_stream; /* hipStream_t */

enum {
  CT_OK = 0,
  CT_E_INVALID = -1,     /* null pointer, non-positive size, bad parameter */
  CT_E_UNSUPPORTED = -2, /* n not of the form 2^a 3^b, n > 8192, ds/h outside [0.75, 1.4] */
  CT_E_DEVICE = -3,      /* a HIP runtime error (message in ct_last_error) */
  CT_E_NONFINITE = -4,   /* validation found NaN/Inf in an input */
  CT_E_DIVERGED = -5,    /* the gap record became non-finite */
  CT_E_STATE = -6        /* call out of order (e.g. gap before any step) */
};

/* Library version (major*10000 + minor*100 + patch). */
int ct_version(void);

/* Message for the last failed call on this thread ("" if none). */
const char *ct_last_error(void);

/* ------------------------------------------------------------------------ */
/* Geometry and projector plan (§3.1 "Discretization")                       */

typedef struct ct_geom {
  int32_t n;        /* image side; n >= 2, n <= 8192 */
  int32_t n_angles; /* N >= 1 */
  int32_t n_bins;   /* M >= 2 */
  double h;         /* pixel spacing > 0 */
  double ds;        /* detector bin width > 0, 0.75 <= ds/h <= 1.4 */
} ct_geom;

typedef struct ct_plan ct_plan;

/* Build the projector plan: per-angle bin-coordinate tables and work lists.
 * angles: HOST array of N radians, or NULL for theta_l = pi l / N.
 * The bin coordinate of pixel (i,j) at angle l is
 *   t = (x_i cos theta_l + y_j sin theta_l)/ds + (M-1)/2,
 * held in 64-bit fixed point with 30 fractional bits (|error| <= (1+i+j) 2^-31),
 * so that R_h and R_h^* use bit-identical interpolation weights.
 * Errors: CT_E_INVALID, CT_E_UNSUPPORTED, CT_E_DEVICE. */
int ct_plan_create(const ct_geom *g, const double *angles, ct_plan **out);

/* Kernel choices fixed at plan creation (ct_plan_create uses all defaults).
 * bp_kernel: the backprojector of standalone ct_radon_adj calls and of
 *   solvers whose tuning is off: CT_BP_AUTO (mirror pairs, 4 pixels per
 *   thread, when at least half of the angles pair as theta, pi - theta, else
 *   one angle at a time), CT_BP_ONE_ANGLE, CT_BP_PAIRS4 or CT_BP_PAIRS8
 *   (CT_E_UNSUPPORTED when the angles do not pair).
 * fwd_angles_per_walk: angles that share one walk of R_h: 0 (4 for n >= 1024
 *   when at least half of the angles form quadruples theta, pi/2 - theta,
 *   pi - theta, pi/2 + theta; else 2 when at least half of them pair up; else
 *   1), 1, 2 or 4 (a mode whose staged windows do not fit falls back to the
 *   next one).  Standalone calls and the solvers' set-up use this walk; a
 *   solver's iteration uses it when it is fixed here, else the one its tuning
 *   chooses (ct_params.fwd_walk). */
enum { CT_BP_AUTO = -1, CT_BP_ONE_ANGLE = 0, CT_BP_PAIRS4 = 4, CT_BP_PAIRS8 = 8 };
typedef struct ct_plan_opts {
  int32_t bp_kernel;
  int32_t fwd_angles_per_walk;
} ct_plan_opts;
/* opts NULL: the defaults (CT_BP_AUTO, 0). */
int ct_plan_create_ex(const ct_geom *g, const double *angles, const ct_plan_opts *opts,
                      ct_plan **out);

/* Host-only self-check of the plan that ct_plan_create would build (no device
 * call): replays the forward projector's fixed-point walk for every strip and
 * staged row and verifies that each LDS read lies in the staged window and
 * that every skipped row holds no pixel of the strip.  *steps (may be NULL)
 * receives the number of (strip, row) steps checked.  CT_E_INVALID with a
 * message naming the strip and row if a check fails. */
int ct_plan_check(const ct_geom *g, const double *angles, int64_t *steps);
/* The same for the plan that ct_plan_create_ex(g, angles, opts) would build. */
int ct_plan_check_ex(const ct_geom *g, const double *angles, const ct_plan_opts *opts,
                     int64_t *steps);
/* out[0] = angles that share one walk of R_h (1, 2 or 4), out[1] = forward-
 * projector groups, out[2] = forward-projector workgroups per problem,
 * out[3] = pixels per thread of the plan's default mirror-pair backprojector
 * (4 or 8; 0: one angle at a time).  Errors: CT_E_INVALID. */
int ct_plan_layout(const ct_plan *p, int32_t out[4]);
int ct_plan_destroy(ct_plan *p);

/* sino = R_h img (§3.1: R_h is the transpose of R_h^*; each pixel's value is
 * split between bins floor(t) and floor(t)+1 with weights 1-alpha and alpha,
 * alpha = t - floor(t); bins outside [0, M) receive nothing).
 * img: [n][n], sino: [N][M] (overwritten).  Ray-driven gather: no atomics,
 * deterministic.  Errors: CT_E_INVALID, CT_E_DEVICE. */
int ct_radon_fwd(const ct_plan *p, const float *img, float *sino, ct_stream s);

/* img = R_h^* sino (§3.1 linear backprojection: per angle the detector row is
 * interpolated linearly at t, values summed over angles; bins outside [0, M)
 * read as zero).  sino: [N][M], img: [n][n] (overwritten).  Pixel-driven
 * gather, deterministic.  Errors: CT_E_INVALID, CT_E_DEVICE. */
int ct_radon_adj(const ct_plan *p, const float *sino, float *img, ct_stream s);

/* p = nabla_h u: forward differences divided by h, zero in the last column
 * (plane 0) and last row (plane 1) (§3.1, Neumann boundary).
 * u: [n][n]; p: [2][n][n] (overwritten). */
int ct_grad(int32_t n, double h, const float *u, float *p, ct_stream s);

/* d = div_h p = -nabla_h^T p: backward differences with Dirichlet boundary
 * (§3.1).  p: [2][n][n]; d: [n][n] (overwritten). */
int ct_div(int32_t n, double h, const float *p, float *d, ct_stream s);

/* ------------------------------------------------------------------------ */
/* Preconditioner (§4.3 periodic Laplacian, §4.3.1 inverse norm, §4.4)       */

typedef struct ct_precond ct_precond;

/* M^{-1} y = F^{-1}( F(y) rho / (sigma^2 c + (sigma tau)^2 lambda_Delta rho) ),
 * rho = sqrt(f1^2 + f2^2 + eps^2) with (f1, f2) the centred integer DFT
 * frequency, lambda_Delta = 4 sin^2(pi k1/n) + 4 sin^2(pi k2/n).
 * n must be 2^a 3^b (mixed-radix FFT in LDS).  sigma, tau, c, eps > 0.
 * Errors: CT_E_INVALID, CT_E_UNSUPPORTED, CT_E_DEVICE. */
int ct_precond_create(int32_t n, double sigma, double tau, double c, double eps,
                      ct_precond **out);
/* x = M^{-1} y; y, x: [n][n] (x may equal y). */
int ct_precond_apply(const ct_precond *m, const float *y, float *x, ct_stream s);
int ct_precond_destroy(ct_precond *m);

/* ------------------------------------------------------------------------ */
/* Pointwise resolvents (§3.3, §4.4), exposed for testing                    */

/* y = (q - s u0)/(1 + s) off D0,  y = min(q - s C, 0) on D0  (count = N*M,
 * row length M for the mask lookup).  mask may be NULL (D0 empty). */
int ct_prox_sino(int32_t n_angles, int32_t n_bins, const float *q, double step,
                 const float *u0, const float *bound, const uint32_t *mask,
                 float *y, ct_stream s);

/* w = q / max(1, |q|/radius) per pixel for a planar field q: [2][n][n]
 * (radius 0 projects onto 0). */
int ct_tv_project(int32_t n, const float *q, double radius, float *w, ct_stream s);

/* ------------------------------------------------------------------------ */
/* Power iteration (§4.3, §5.1)                                             */

/* *out = sqrt(lambda_max(R_h^* R_h)) by `iters` steps x <- R^*R x/||R^*R x||
 * from x0 (device [n][n]; NULL: a fixed deterministic start), the estimate
 * being ||R^*R x|| at the last step.  Norms reduced in FP64.  Synchronizes s. */
int ct_power_norm(const ct_plan *p, int32_t iters, const float *x0, double *out,
                  ct_stream s);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * power iteration as ct_power_norm, with its work image, sinogram and FP64
 * reduction partials in a 64 MiB array that the library holds on each device
 * it runs on (for the life of the process) instead of the plan's scratch.  It
 * calls no allocating routine: the array is looked up (and so loaded by the
 * runtime) on a device when the first plan is created there.  Its backprojections run with one angle
 * slice, so the estimate agrees with ct_power_norm's to FP32 rounding.
 * Limit: 4 (n^2 + N M) bytes plus 12 KiB of partials must fit the array
 * (n^2 + N M up to about 16.7 million; CT_E_INVALID beyond).  x0 (device
 * [n][n], not modified) or NULL for ct_power_norm's default start.  Calls
 * on one device share the array: calls that overlap in time on one device
 * (other host threads, other streams) race and must be serialized by the
 * caller.  Synchronizes s.  Errors: CT_E_INVALID, CT_E_UNSUPPORTED,
 * CT_E_DEVICE. */
int ct_power_norm_noalloc(const ct_plan *p, int32_t iters, const float *x0, double *out,
                          ct_stream s);

/* ------------------------------------------------------------------------ */
/* Solver: problem setup and Algorithm PDRQS1                               */

typedef struct ct_problem {
  const float *sino;     /* u0: [N][M] measured sinogram (device) */
  const uint32_t *mask;  /* D0 bitmask [N][ceil(M/32)] (device) or NULL (D0 empty) */
  const float *bound;    /* C: [N][M] (device) or NULL to use bound_scalar */
  float bound_scalar;    /* C when bound is NULL */
  float pad_;
  double lambda;         /* lambda of (C_h) (unnormalized), >= 0 */
} ct_problem;

enum {
  CT_FLAG_VALIDATE = 1u, /* scan sino/bound for NaN/Inf at setup (CT_E_NONFINITE) */
  CT_METHOD_SHIFT = 4u,  /* flags bits 4..7 select the iteration (CT_METHOD_*) */
  CT_FLAG_NONNEG = 2u    /* add u >= 0 (§4.5): the iteration gains the state bar u,
                            u_tmp = bar u - u - sigma (A^* s1 - tau div s2), the
                            multiplier rho / (rho + sigma^2 c + (sigma tau)^2 lambda_Delta rho),
                            and bar u += max(2 u_new - bar u, 0) - u_new */
};

/* Iterations a solver can run (flags |= method << CT_METHOD_SHIFT):
 *  PDRQS1      Algorithm PDRQS1 (§4.4), inverse-norm + periodic-Laplacian M (default)
 *  RICHARDSON  PDRQS1 with M = m id, m = 1.1 (sigma^2 + 8 (sigma tau)^2 / h^2) (§4.3)
 *  CP          Algorithm CP (§3.4), sigma = tau = 0.99 / sqrt(1 + 8/h^2) on the
 *              normalized problem (the params' sigma, tau are not used)
 *  PDRQS2      Algorithm PDRQS2 (§4.2, §4.3.1), the unconstrained problem (no D0)
 *  ADMM        ADMM with an inner PCG u-step (§4.6), the unconstrained problem
 *              (no D0), one problem per solver; see ct_solver_set_admm
 *  PDRQS3      PDRQS1's iteration with the splitting PDRQ3 of §4.4's table: the
 *              fit's quadratic part in the dual (S = diag(chi_{D\D0}, 0), g = (b, 0)):
 *              u_tmp = -sigma (A^* s1 - tau div s2) with s1 = D (vb1 + sigma (A u - g)),
 *              D = 1/(1 + sigma) off D0; off D0 vb1 <- (vb1 + sigma (A u_new - b)) /
 *              (1 + sigma), on D0 the constraint's resolvent as in PDRQS1
 * ct_gap is defined for PDRQS1 and RICHARDSON; ct_objective serves all. */
/* Preconditioner of PDRQS1 (flags |= kind << CT_PRECOND_SHIFT):
 *  INVNORM   inverse norm + periodic Laplacian (§4.3.1): rho / (sigma^2 c +
 *            (sigma tau)^2 lambda_Delta rho), c = c_safety lambda_max(tilde M^{-1} A^* A)
 *  IMPULSE   impulse response (§4.3.2): k = the response of A^* A to a unit
 *            impulse at (n/2, n/2), centred at the origin and averaged over the
 *            symmetries of the square; K = sigma^2 k + (sigma tau)^2 kappa_Delta;
 *            M = c F^{-1} F(K) F with c = c_safety lambda_max(M_K^{-1} T) (even n;
 *            CT_E_UNSUPPORTED if F(K) is not positive or for other methods)
 *  CIRCULANT circulant approximation (§4.3.3): on the column-major vectorized
 *            image (index j + n i), the response of A^* A shifted to index 0 and
 *            symmetrized as the circulant's first column, K = sigma^2 k + (sigma
 *            tau)^2 kappa_Delta, M = c F_L^{-1} F_L(K) F_L with the length-n^2 DFT
 *            and c as for IMPULSE (same restrictions)
 * IMPULSE and CIRCULANT: one problem per solver. */
enum {
  CT_PRECOND_SHIFT = 8u,
  CT_PRECOND_INVNORM = 0,
  CT_PRECOND_IMPULSE = 1,
  CT_PRECOND_CIRCULANT = 2
};

enum {
  CT_METHOD_PDRQS1 = 0,
  CT_METHOD_RICHARDSON = 1,
  CT_METHOD_CP = 2,
  CT_METHOD_PDRQS2 = 3,
  CT_METHOD_ADMM = 4,
  CT_METHOD_PDRQS3 = 5
};

typedef struct ct_params {
  double sigma;          /* PDRQ step sigma > 0 (default 1) */
  double tau;            /* gradient scaling tau > 0 (default 1/sqrt(8)) */
  double eps;            /* inverse-norm regularization eps > 0 (default 0.3) */
  double c;              /* preconditioner constant; <= 0: c_safety * power-iteration estimate */
  double c_safety;       /* default 1.1 */
  double beta;           /* normalization ||R_h||; <= 0: power-iteration estimate */
  int32_t k_max;         /* iterations for ct_reconstruct, >= 0 */
  int32_t gap_every;     /* gap record period for ct_reconstruct (0: none) */
  int32_t power_iters;   /* power-iteration steps (default 30) */
  uint32_t flags;        /* CT_FLAG_* */
  const float *start_norm;    /* device [n][n] start of the ||R_h|| iteration or NULL */
  const float *start_precond; /* device [n][n] start of the c iteration or NULL */
  /* Launch choices of the iteration.  0 in each field: chosen by the
   * solver's set-up tuning (or the plan's defaults with CT_OPT_NO_TUNE). */
  int32_t bp_slices;     /* angle slices of R_h^* (1..16), 0: tuned */
  int32_t bp_kernel;     /* CT_BP_* backprojector of the iteration; CT_BP_AUTO: tuned */
  int32_t tv_blocks;     /* workgroups of the gradient-side update inside R_h's launch
                            (1..4096), 0: tuned */
  uint32_t options;      /* CT_OPT_* */
  const char *tune_cache; /* path of a JSON file of tuning results, or NULL.  A choice
                            found there (same GPU, geometry, batch size, method) is
                            used without timing; a new one is added to the file.
                            Reusing the file makes the launch choices, and so the
                            FP32 summation order, the same in every process. */
  int32_t fwd_walk;      /* angles per walk of R_h in the iteration: 1, 2 or 4 (a mode
                            whose staged windows do not fit falls back as in
                            ct_plan_opts), 0: the plan's walk when its
                            fwd_angles_per_walk was fixed, else tuned.  A walk other
                            than the plan's gets forward tables of the solver's own. */
} ct_params;

/* ct_params.options bits. */
enum {
  CT_OPT_NO_TUNE = 1u,     /* no timing at set-up: the plan's walk and backprojector, its
                              default slice count and 256 gradient-side workgroups (unless
                              fixed) */
  CT_OPT_NO_DEFER = 2u,    /* sum R_h^*'s angle slices in a pass of its own, not in the
                              preconditioner's first FFT pass (same arithmetic) */
  CT_OPT_SEPARATE_TV = 4u, /* run the gradient-side update as its own launch (same
                              arithmetic) */
  CT_OPT_NO_GRAPH = 8u     /* launch the iterations one by one, no HIP graph */
};

/* Fill *p with the defaults above (k_max = 0, gap_every = 0, bp_slices = 0,
 * bp_kernel = CT_BP_AUTO, tv_blocks = 0, options = 0, tune_cache = NULL,
 * fwd_walk = 0). */
void ct_params_default(ct_params *p);

/* Objective of (C_h) at u [n][n] (device), in the problem's units (§3.2):
 * out[0] = 1/2 sum_{D\D0} (R_h u - u0)^2, out[1] = lambda ||nabla_h u||_1,
 * out[2] = max_{D0} (C - R_h u)_+ (the constraint violation).  FP64 sums.
 * Uses the plan's scratch; synchronizes s. */
int ct_objective(const ct_plan *p, const ct_problem *prob, const float *u, double out[3],
                 ct_stream s);

/* Metal-trace estimate from a reconstruction (results chapter, real metal
 * artifacts): the pixels of u_rec above `threshold` are marked, the marks are
 * dilated by the disk {a^2 + b^2 <= radius^2} of pixel offsets, the dilated
 * indicator chi is projected, and D0 holds the bins with (R_h chi) > kappa
 * (kappa >= 0: the smallest interpolation weight with which a marked pixel
 * must reach a bin; the two weights of a pixel sum to 1).  When u0 and bound
 * are given, bound = c0 u0 on D0 and 0 elsewhere (the thesis takes c0 = 0.8).
 * u_rec: device [n][n]; chi: device [n][n] out (0 or 1); proj: device [N][M]
 * out; mask: device uint32 [N][ceil(M/32)] out, bit k & 31 of word k >> 5;
 * u0, bound: device [N][M] (both NULL or both non-NULL).  Buffers are the
 * caller's; nothing is allocated.  0 <= radius <= 16.
 * Errors: CT_E_INVALID (null or out-of-range argument), CT_E_DEVICE. */
int ct_d0_estimate(const ct_plan *p, const float *u_rec, float threshold, int32_t radius,
                   float kappa, float *chi, float *proj, uint32_t *mask, const float *u0,
                   float c0, float *bound, ct_stream s);

typedef struct ct_solver ct_solver;

/* Setup (§5.1, §4.3.1): beta (power iteration unless given), data b = u0/beta,
 * bounds C/beta, lambda~ = lambda/beta^2, c (power iteration on
 * tilde M^{-1/2} A^*A tilde M^{-1/2} unless given), the Fourier multiplier,
 * and a zero state u = bar v1 = bar v2 = 0.  The solver keeps pointers to
 * problem->sino/mask/bound only during this call (it copies what it needs).
 * Synchronizes s.  Errors: CT_E_INVALID, CT_E_UNSUPPORTED, CT_E_NONFINITE,
 * CT_E_DEVICE. */
int ct_solver_create(const ct_plan *p, const ct_problem *prob, const ct_params *prm,
                     ct_stream s, ct_solver **out);

/* A solver for nb >= 1 problems of the plan's geometry (probs[0..nb-1], all
 * with the same lambda), advanced together: every kernel of an iteration
 * covers the nb problems in one launch.  beta and c depend on the geometry
 * only and are estimated once.  The backprojector, its number of angle
 * slices and the gradient-side update's workgroups are tuned at set-up by
 * timing the candidates on the batch, unless fixed by the params (see
 * ct_params.bp_slices ... options, tune_cache; ct_solver_tuning reports how
 * the choice was made).  All state arrays of the other calls then hold nb problems
 * one after the other ([nb][n][n], [nb][N][M], [nb][2][n][n]); ct_gap writes
 * 6 doubles per problem.  Errors as ct_solver_create. */
int ct_solver_create_batch(const ct_plan *p, const ct_problem *probs, int32_t nb,
                           const ct_params *prm, ct_stream s, ct_solver **out);
int ct_solver_destroy(ct_solver *sv);

/* out[0] = beta, out[1] = c, out[2] = lambda~, out[3] = iterations done. */
int ct_solver_info(const ct_solver *sv, double out[4]);

/* How the solver's launch choices were made: out[0] = 0 fixed by the
 * params or CT_OPT_NO_TUNE, 1 timed at set-up, 2 taken from an earlier solver
 * of the same plan, batch size and method class, 3 read from the tune cache
 * file; out[1] = candidate launches timed by this solver (0 unless out[0] is
 * 1); out[2] = workgroups of the gradient-side update inside R_h's launch
 * (0: a separate launch); out[3] = 1 if the choice was added to the tune
 * cache file. */
int ct_solver_tuning(const ct_solver *sv, int32_t out[4]);

/* out[0] = problems in the solver, out[1] = angle slices of R_h^*,
 * out[2] = angles that share one walk in R_h's iteration launches (1, 2 or
 * 4; chosen by the solver's tuning unless fixed),
 * out[3] = forward-projector groups of that walk,
 * out[4] = angles that share one bin coordinate in R_h^* (2: mirror pairs
 * theta, pi - theta; 1: one angle at a time; chosen by the solver's tuning),
 * out[5] = pixels per thread of the mirror-pair kernel (4 or 8; 0 without). */
int ct_solver_layout(const ct_solver *sv, int32_t out[6]);

/* Data-term variants of §3.5 for PDRQS1 (and its Richardson form), set before
 * the first iteration:
 *  STANDARD    1/2 (A u - b)^2 off D0, C~ <= A u on D0 (default)
 *  WEIGHTED    1/2 w (A u - b)^2 off D0; aux = w [nb][N][M] (device, w > 0)
 *  IGNORE      no term on D0 (the bound is not used)
 *  EVERYWHERE  1/2 (A u - b)^2 on every bin plus C~ <= A u on D0;
 *              aux = u0 [nb][N][M] (device, unnormalized) including D0
 *  HARD        A u = b off D0, C~ <= A u on D0
 * ct_gap and the reverse sweep are defined for STANDARD only.  Errors:
 * CT_E_STATE after the first iteration, CT_E_UNSUPPORTED for other methods. */
enum {
  CT_FIT_STANDARD = 0,
  CT_FIT_WEIGHTED = 1,
  CT_FIT_IGNORE = 2,
  CT_FIT_EVERYWHERE = 3,
  CT_FIT_HARD = 4
};
int ct_solver_set_fit(ct_solver *sv, int32_t fit, const float *aux, ct_stream s);

/* ADMM options (§4.6) of a CT_METHOD_ADMM solver, before its first iteration:
 * cg_steps in [1, 64] preconditioned conjugate-gradient steps per iteration on
 * (A^* A - tau^2 Delta_h) u = A^*(z_w - eta_w) - tau^2 div(z_v - eta_v), started
 * from the current u, preconditioned by rho_eps / (c + tau^2 lambda_Delta
 * rho_eps) (§4.3.1); the augmented-Lagrangian weight mu > 0 (Lambda = diag(1,
 * tau) weights the gradient block).  One iteration: the PCG u-step, then
 * w = (b + mu (A u + eta_w)) / (1 + mu), v = soft(nabla u + eta_v,
 * lambda~ / (mu tau^2)), eta <- eta - (z - K u).  Defaults: 1 step, mu = 1.
 * The solver's state export gives (u, eta_w, eta_v).
 * Errors: CT_E_INVALID, CT_E_UNSUPPORTED (not an ADMM solver), CT_E_STATE
 * (after the first iteration). */
int ct_solver_set_admm(ct_solver *sv, int32_t cg_steps, double mu);

/* Run k iterations of PDRQS1 (§4.4) on the solver's state:
 *   u_tmp = -sigma (A^*(vb1 + sigma A u) - tau div(vb2 + sigma tau nabla u))
 *   u     = u + M^{-1} u_tmp
 *   v1 = vb1 + sigma A u,  v2 = vb2 + sigma tau nabla u
 *   y1 = prox_sino(2 v1 - vb1, sigma),   vb1 += y1 - v1
 *   w  = tv_project(2 v2 - vb2, lambda~/tau),  vb2 += w - v2
 * A u and nabla u are cached across iterations (one R_h and one R_h^* per
 * iteration).  Asynchronous; k >= 0. */
int ct_pd_step(ct_solver *sv, int32_t k, ct_stream s);

/* Same iterations as ct_pd_step (k >= 1), with the same launches, launched
 * one by one with HIP events on s around each phase; ms_out receives the
 * average duration per iteration in milliseconds of [0] R_h^* with the u_tmp
 * epilogue, [1] the preconditioner update u + M^{-1} u_tmp (§4.3.1), [2] R_h
 * with the sinogram-side update (and the gradient-side update when that runs
 * in R_h's launch), [3] the gradient-side update when it is a launch of its
 * own (else about 0), [4] their sum.  Synchronizes s after every iteration,
 * so it measures kernels, not throughput.  The state advances as with
 * ct_pd_step. */
int ct_pd_step_timed(ct_solver *sv, int32_t k, double ms_out[5], ct_stream s);

/* Copy the state out: u [n][n], vb1 [N][M], vb2 [2][n][n] (any may be NULL). */
int ct_state_export(const ct_solver *sv, float *u, float *vb1, float *vb2, ct_stream s);
/* bar u of the non-negativity variant ([nb][n][n]); CT_E_STATE without it. */
int ct_state_export_ubar(const ct_solver *sv, float *ubar, ct_stream s);
int ct_state_import_ubar(ct_solver *sv, const float *ubar, ct_stream s);
/* Replace the state (all three required); caches A u, nabla u are recomputed. */
int ct_state_import(ct_solver *sv, const float *u, const float *vb1, const float *vb2,
                    ct_stream s);

/* FP64 record of the current state, in normalized units, with y = (y1, w)
 * the resolvent outputs of the last iteration:
 *   out[0] P  = 1/2 sum_{D\D0} (A u - b)^2 + lambda~ sum |nabla u|
 *   out[1] G* = sum_{D\D0} (y1^2/2 + y1 b) + sum_{D0} y1 C~
 *   out[2] gap = P + G*
 *   out[3] ||A^* y1 - tau div w||
 *   out[4] max_{D0} (C~ - A u)_+
 *   out[5] ||u_k - u_{k-1}||
 * (6 doubles per problem for a batch solver, in problem order)
 * Requires at least one ct_pd_step since creation/import (CT_E_STATE).
 * Synchronizes s. */
int ct_gap(ct_solver *sv, double *out, ct_stream s);

/* One-shot solve: setup, k_max iterations, u_out [n][n].  With gap_every > 0
 * and report non-NULL, writes 6 doubles per record into report (capacity
 * report_len doubles, records after iterations gap_every, 2 gap_every, ...).
 * Returns CT_E_DIVERGED if a record is non-finite.  Synchronizes s. */
int ct_reconstruct(const ct_plan *p, const ct_problem *prob, const ct_params *prm,
                   float *u_out, double *report, int32_t report_len, ct_stream s);

typedef struct ct_group ct_group;

/* A group of solvers (any geometries, same number of iterations done) that
 * ct_group_step advances together: k iterations of every solver, all but the
 * last replayed from one HIP graph holding two iterations of every solver.
 * The group does not own the solvers; destroy it before them.  A solver
 * stepped on its own afterwards makes ct_group_step fail with CT_E_STATE. */
int ct_group_create(ct_solver *const *svs, int32_t count, ct_group **out);
int ct_group_step(ct_group *g, int32_t k, ct_stream s);
int ct_group_destroy(ct_group *g);

/* count problems, problem i on plans[i] (any mix of geometries), output
 * u_out[i] [n_i][n_i] (device).  Problems with the same plan and lambda are
 * advanced as one batch (ct_solver_create_batch); the iterations of all
 * batches are captured together in one HIP graph and replayed.  Report
 * layout: report[(i * R + r) * 6 + q] for record r < R = k_max / gap_every
 * (records that do not fit report_len are skipped).  Synchronizes s. */
int ct_reconstruct_batched(int32_t count, const ct_plan *const *plans, const ct_problem *probs,
                           const ct_params *prm, float *const *u_out, double *report,
                           int32_t report_len, ct_stream s);

/* Differentiation through K unrolled PDRQS1 iterations (§4.4 applied K
 * times from the zero state).  ct_unrolled_forward resets the solver's state,
 * runs K iterations (graph-replayed) and keeps the state every `every`
 * iterations in the returned tape; u_K is then the solver's state
 * (ct_state_export).  Synchronizes s.
 * ct_unrolled_backward takes gbar = dL/du_K (device, the solver's [nb][n][n]
 * layout) and returns dL/du0 (device [nb][N][M], zero on the metal trace,
 * may be NULL) and dL/dlambda per problem (host, nb doubles, may be NULL),
 * by the reverse sweep of the iteration: each segment between checkpoints is
 * recomputed once, then swept backwards through the transposed linear maps
 * (A, A^*, nabla, div, M^{-1}) and the Jacobians of the two resolvents.  beta
 * and c are held fixed (they depend on the geometry only).  It leaves the
 * solver's state undefined; the tape stays valid for further backward calls
 * as long as the solver is not stepped.  Synchronizes s.  The tape borrows the
 * solver: destroy the tape first. */
typedef struct ct_tape ct_tape;
int ct_unrolled_forward(ct_solver *sv, int32_t K, int32_t every, ct_tape **out, ct_stream s);
int ct_unrolled_backward(ct_tape *t, const float *gbar, float *grad_u0, double *grad_lambda,
                         ct_stream s);
int ct_tape_destroy(ct_tape *t);

/* ------------------------------------------------------------------------ */
/* Measurement utilities (not steps of the method)                           */

/* A probe of the vector issue rate: `blocks` workgroups of 256 threads whose
 * lanes each run 16 independent chains for `iters` rounds, i.e.
 * blocks * 4 * iters * 16 * I wave-instructions of 64 lanes, by kind:
 * 0 FP32 FMA (I = 1), 1 FP32 add (I = 1), 2 32-bit integer xor-add (I = 1),
 * 3 integer xor-add and integer-to-float conversion (I = 2), 4 64-bit
 * integer add (I = 1).  Timed with
 * events on s, it gives the achievable VALU rate of each kind, against which
 * the projectors' issue fractions are read.  out: device buffer of `blocks`
 * floats, written only if a chain turned negative (never; the store keeps
 * the work live).  Asynchronous.  Errors: CT_E_INVALID, CT_E_DEVICE. */
int ct_valu_probe(int32_t blocks, int32_t iters, int32_t kind, float *out, ct_stream s);

/* A streaming copy of `bytes` bytes (a positive multiple of 16) between two
 * non-overlapping, 16-byte aligned device buffers by `blocks` workgroups of
 * 256 threads with 16-byte accesses.  Timed with events on s over buffers
 * larger than the 256 MB last-level cache, it gives the achievable HBM
 * bandwidth (2 * bytes moved).  Asynchronous.  Errors: CT_E_INVALID,
 * CT_E_DEVICE. */
int ct_copy_probe(const void *src, void *dst, int64_t bytes, int32_t blocks, ct_stream s);

#ifdef __cplusplus
}
#endif

#endif /* CTPD_H */
