// C ABI of ctpd: argument validation, object lifetimes and the PDRQS1 driver
// (thesis Algorithm PDRQS1 in §4.4, setup of §5.1 and §4.3.1).
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <new>
#include <type_traits>
#include <string>
#include <vector>

#include <unistd.h>

#include "common.hpp"

namespace ctpd {

static thread_local std::string g_err;
void set_error(const std::string &msg) { g_err = msg; }
void clear_error() { g_err.clear(); }

int build_plan(const ct_geom *g, const double *angles, const ct_plan_opts &opt, ct_plan *p);
int build_fwd_plan(const ct_plan *base, int walk, ct_plan *p);
int check_plan(const ct_geom *g, const double *angles, const ct_plan_opts &opt, int64_t *steps);
void free_plan(ct_plan *p);
int noalloc_prepare_device();

static bool fft_size_ok(int n) {
  if (n < 2 || n > 4096 || (n & 1)) return false;
  int m = n;
  while (m % 2 == 0) m /= 2;
  while (m % 3 == 0) m /= 3;
  return m == 1;
}

static hipStream_t S(ct_stream s) { return reinterpret_cast<hipStream_t>(s); }

// ---------------------------------------------------------------------------
// Preconditioner tables (§4.3, §4.3.1, §4.4), computed in FP64 on the host.
static double freq(int k, int n) { return (k <= n / 2) ? (double)k : (double)(k - n); }

// sqrt_rho_only: sqrt(rho) (the c estimate); nonneg: the u >= 0 variant's
// rho / (rho + sigma^2 c + (sigma tau)^2 lambda_Delta rho) (§4.5).
static std::vector<float> multiplier_table(int n, double sigma, double tau, double c, double eps,
                                           bool sqrt_rho_only, bool nonneg = false) {
  const int half = n / 2 + 1;
  std::vector<float> m((size_t)half * n);
  const double inv_nn = 1.0 / ((double)n * (double)n);
  for (int k1 = 0; k1 < half; ++k1) {
    const double s1 = std::sin(M_PI * k1 / n);
    const double f1 = freq(k1, n);
    for (int k2 = 0; k2 < n; ++k2) {
      const double s2 = std::sin(M_PI * k2 / n);
      const double f2 = freq(k2, n);
      const double rho = std::sqrt(f1 * f1 + f2 * f2 + eps * eps);
      double v;
      if (sqrt_rho_only) {
        v = std::sqrt(rho);
      } else {
        const double lap = 4.0 * s1 * s1 + 4.0 * s2 * s2;
        v = rho / ((nonneg ? rho : 0.0) + sigma * sigma * c +
                   (sigma * tau) * (sigma * tau) * lap * rho);
      }
      m[(size_t)k1 * n + k2] = (float)(v * inv_nn);
    }
  }
  return m;
}

static int precond_init(ct_precond *pc, int n, double sigma, double tau, double c, double eps) {
  pc->n = n;
  pc->sigma = sigma;
  pc->tau = tau;
  pc->c = c;
  pc->eps = eps;
  if (!fft_factor(n, &pc->fp)) {
    set_error("FFT size must be 2^a 3^b");
    return CT_E_UNSUPPORTED;
  }
  std::vector<float2> tw(n);
  for (int m = 0; m < n; ++m) {
    const double a = -2.0 * M_PI * (double)m / (double)n;
    tw[m] = make_float2((float)std::cos(a), (float)std::sin(a));
  }
  const int half = n / 2 + 1;
  CT_TRY_HIP(hipMalloc(&pc->d_tw, sizeof(float2) * n));
  CT_TRY_HIP(hipMemcpy(pc->d_tw, tw.data(), sizeof(float2) * n, hipMemcpyHostToDevice));
  CT_TRY_HIP(hipMalloc(&pc->d_spec, sizeof(float2) * (size_t)half * n));
  CT_TRY_HIP(hipMalloc(&pc->d_mult, sizeof(float) * (size_t)half * n));
  if (c > 0) {
    auto m = multiplier_table(n, sigma, tau, c, eps, false);
    CT_TRY_HIP(hipMemcpy(pc->d_mult, m.data(), sizeof(float) * m.size(), hipMemcpyHostToDevice));
  }
  return CT_OK;
}

static void precond_free(ct_precond *pc) {
  (void)hipFree(pc->d_tw);
  (void)hipFree(pc->d_spec);
  (void)hipFree(pc->d_mult);
  pc->d_tw = nullptr;
  pc->d_spec = nullptr;
  pc->d_mult = nullptr;
}

// Scratch owned by a plan for standalone calls (allocated on first use).
static int plan_scratch(ct_plan *p) {
  const size_t nn = (size_t)p->g.n * p->g.n, NM = (size_t)p->g.n_angles * p->g.n_bins;
  if (!p->d_scratch_img) CT_TRY_HIP(hipMalloc(&p->d_scratch_img, sizeof(float) * nn * 2));
  if (!p->d_scratch_sino) CT_TRY_HIP(hipMalloc(&p->d_scratch_sino, sizeof(float) * NM));
  if (!p->d_red) {
    p->red_cap = reduction_partials_needed() + 16;
    CT_TRY_HIP(hipMalloc(&p->d_red, sizeof(double) * p->red_cap));
  }
  return CT_OK;
}

static std::vector<float> default_start(int n) {
  // smooth, non-symmetric, non-zero-mean start image
  std::vector<float> x((size_t)n * n);
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i)
      x[(size_t)j * n + i] = (float)(1.0 + 0.5 * std::sin(0.37 * i + 1.13 * j) +
                                     0.25 * std::cos(0.071 * i * j + 0.3));
  return x;
}

// lambda_max of op by `iters` power steps; x is a work image holding the start.
// op(x, y) computes y = op(x).  Norms in FP64 on the device.
template <class Op>
static int power_iterate(int n, int iters, float *x, float *y, double *d_red, int red_cap,
                         double *d_norm, Op op, hipStream_t s, double *lam_out) {
  const int64_t nn = (int64_t)n * n;
  CT_TRY(launch_norm2(x, nn, d_red, red_cap, d_norm, s));
  CT_TRY(launch_scale_by_inv(x, nn, d_norm, x, s));
  for (int it = 0; it < iters; ++it) {
    CT_TRY(op(x, y));
    CT_TRY(launch_norm2(y, nn, d_red, red_cap, d_norm, s));
    CT_TRY(launch_scale_by_inv(y, nn, d_norm, x, s));
  }
  double lam = 0.0;
  CT_TRY_HIP(hipMemcpyAsync(&lam, d_norm, sizeof(double), hipMemcpyDeviceToHost, s));
  CT_TRY_HIP(hipStreamSynchronize(s));
  *lam_out = lam;
  return CT_OK;
}

}  // namespace ctpd

using namespace ctpd;

// Cached iteration graphs per ping-pong parity: [parity] two iterations,
// [2 + parity] two iterations whose last keeps y1, w and A u for a record,
// [4 + parity] 2 kLongPairs iterations (the bulk of a long run in one launch).
constexpr int kGraphSlots = 6;
constexpr int kLongPairs = 8;

struct ct_solver {
  ct_plan *plan = nullptr;
  ct_precond pc{};
  int nb = 1;  // problems advanced together
  int n = 0, N = 0, M = 0;
  double beta = 0, c = 0, lam_t = 0, sigma = 0, tau = 0, eps = 0;
  float *u = nullptr, *u_next = nullptr, *vb1 = nullptr, *s1 = nullptr, *vb2 = nullptr,
        *s2 = nullptr, *target = nullptr, *rraw = nullptr, *utmp = nullptr;
  float *y1 = nullptr, *r = nullptr, *w = nullptr;
  uint32_t *mask = nullptr;
  float2 *spec = nullptr;     // nb spectra of the preconditioner FFT
  float *bp_part = nullptr;   // nb * bp_S partial backprojections
  float *ubar = nullptr;      // bar u of the u >= 0 variant (nb images) or NULL
  int method = 0;             // CT_METHOD_*
  float *ucp = nullptr;       // Algorithm CP: the extrapolated iterate (nb images)
  double rich_m = 0;          // Richardson: M = rich_m id
  int fit = 0;                // data-term variant (CT_FIT_*)
  float *fit_aux = nullptr;   // its per-bin array (nb sinograms) or NULL
  // ADMM (§4.6): vb1, vb2 hold eta_w, eta_v; s1, s2 the u-step residual terms
  // (z_w - eta_w) - A u and (z_v - eta_v) - nabla u; PCG vectors and scalars
  int admm_cg = 1;
  double admm_mu = 1.0;
  float *cg_r = nullptr, *cg_z = nullptr, *cg_p = nullptr, *cg_Hp = nullptr;
  double *d_cg = nullptr;     // [0], [1] r.z (alternating), [2] p.Hp, then dot partials
  bool defer_combine = true;  // form R_h^*'s slice sum in the FFT row pass
  bool fuse_tv = true;        // run the gradient-side update in R_h's launch
  size_t bp_cap = 0;
  int bp_S = 1;               // angle slices of the backprojection (tuned)
  int bp_kern = 4;            // backprojector of the iteration (0 one angle, 4 or 8 pairs)
  int tv_blocks = 256;        // gradient-side workgroups in R_h's launch (0: own launch)
  // R_h of the iteration: the plan itself, or forward tables of the solver's
  // own for another number of angles per walk (fwd_alt, built for fwd_alt_walk)
  const ct_plan *fwd = nullptr;
  ct_plan *fwd_alt = nullptr;
  int fwd_alt_walk = 0;
  uint32_t options = 0;       // CT_OPT_*
  // how the launch choices were made (ct_solver_tuning)
  int tune_source = 0, tune_timed = 0, tune_saved = 0;
  double *d_red = nullptr, *d_out = nullptr;
  int red_cap = 0;
  int64_t iters = 0;
  bool have_dual = false;
  // Two PDRQS1 iterations captured as a HIP graph, one per ping-pong parity of
  // (u, u_next); captured on a private stream, replayed on the caller's stream.
  hipStream_t cap_stream = nullptr;
  // index parity + 2 * (the second iteration keeps y1, w and A u for a record)
  hipGraphExec_t gexec[kGraphSlots] = {};
  float *gexec_u[kGraphSlots] = {};
  bool use_graph = true;
};

static bool has_graphs(const ct_solver *sv) {
  for (auto g : sv->gexec)
    if (g) return true;
  return false;
}

static void solver_free(ct_solver *sv) {
  if (!sv) return;
  float *bufs[] = {sv->u, sv->u_next, sv->vb1, sv->s1, sv->vb2, sv->s2, sv->target,
                   sv->rraw, sv->utmp, sv->y1, sv->r, sv->w, sv->bp_part, sv->ubar, sv->ucp,
                   sv->fit_aux, sv->cg_r, sv->cg_z, sv->cg_p, sv->cg_Hp};
  for (float *b : bufs) (void)hipFree(b);
  (void)hipFree(sv->mask);
  (void)hipFree(sv->spec);
  (void)hipFree(sv->d_red);
  (void)hipFree(sv->d_out);
  (void)hipFree(sv->d_cg);
  for (auto &g : sv->gexec)
    if (g) (void)hipGraphExecDestroy(g);
  if (sv->cap_stream) (void)hipStreamDestroy(sv->cap_stream);
  precond_free(&sv->pc);
  if (sv->fwd_alt) {
    free_plan(sv->fwd_alt);
    delete sv->fwd_alt;
    sv->fwd_alt = nullptr;
  }
}

extern "C" {

int ct_version(void) { return 10100; }

const char *ct_last_error(void) { return g_err.c_str(); }

void ct_params_default(ct_params *p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->sigma = 1.0;
  p->tau = 1.0 / std::sqrt(8.0);
  p->eps = 0.3;
  p->c = 0.0;
  p->c_safety = 1.1;
  p->beta = 0.0;
  p->k_max = 0;
  p->gap_every = 0;
  p->power_iters = 30;
  p->flags = 0;
  p->bp_slices = 0;
  p->bp_kernel = CT_BP_AUTO;
  p->tv_blocks = 0;
  p->options = 0;
  p->tune_cache = nullptr;
  p->fwd_walk = 0;
}

static int check_geom(const ct_geom *g, const double *angles) {
  if (g->n < 2 || g->n_angles < 1 || g->n_bins < 2 || !(g->h > 0) || !(g->ds > 0)) {
    set_error("ct_plan_create: need n >= 2, N >= 1, M >= 2, h > 0, ds > 0");
    return CT_E_INVALID;
  }
  if (g->n > 8192 || g->n_bins > (1 << 20) || g->n_angles > (1 << 20)) {
    set_error("ct_plan_create: size too large (n <= 8192)");
    return CT_E_UNSUPPORTED;
  }
  const double ratio = g->ds / g->h;
  if (ratio < 0.75 || ratio > 1.4) {
    set_error("ct_plan_create: ds/h must lie in [0.75, 1.4]");
    return CT_E_UNSUPPORTED;
  }
  if (angles) {
    for (int l = 0; l < g->n_angles; ++l)
      if (!std::isfinite(angles[l])) {
        set_error("ct_plan_create: non-finite angle");
        return CT_E_INVALID;
      }
  }
  return CT_OK;
}

static int check_opts(const ct_plan_opts *o, ct_plan_opts *out) {
  *out = ct_plan_opts{CT_BP_AUTO, 0};
  if (!o) return CT_OK;
  if ((o->bp_kernel != CT_BP_AUTO && o->bp_kernel != CT_BP_ONE_ANGLE &&
       o->bp_kernel != CT_BP_PAIRS4 && o->bp_kernel != CT_BP_PAIRS8) ||
      o->fwd_angles_per_walk < 0 || o->fwd_angles_per_walk > 4 || o->fwd_angles_per_walk == 3) {
    set_error("ct_plan_create: bp_kernel must be a CT_BP_* value, fwd_angles_per_walk 0, 1, 2 "
              "or 4");
    return CT_E_INVALID;
  }
  *out = *o;
  return CT_OK;
}

int ct_plan_create(const ct_geom *g, const double *angles, ct_plan **out) {
  return ct_plan_create_ex(g, angles, nullptr, out);
}

int ct_plan_create_ex(const ct_geom *g, const double *angles, const ct_plan_opts *opts,
                      ct_plan **out) {
  clear_error();
  if (!g || !out) {
    set_error("ct_plan_create: null argument");
    return CT_E_INVALID;
  }
  *out = nullptr;
  CT_TRY(check_geom(g, angles));
  ct_plan_opts opt;
  CT_TRY(check_opts(opts, &opt));
  ct_plan *p = new (std::nothrow) ct_plan();
  if (!p) return CT_E_DEVICE;
  p->g = *g;
  (void)hipGetDevice(&p->device);
  int rc = build_plan(g, angles, opt, p);
  if (rc == CT_OK) rc = noalloc_prepare_device();
  if (rc != CT_OK) {
    free_plan(p);
    delete p;
    return rc;
  }
  *out = p;
  return CT_OK;
}

int ct_plan_layout(const ct_plan *p, int32_t out[4]) {
  clear_error();
  if (!p || !out) {
    set_error("ct_plan_layout: null argument");
    return CT_E_INVALID;
  }
  out[0] = p->slots;
  out[1] = p->n_groups;
  out[2] = p->n_work;
  out[3] = p->bp_kern0;
  return CT_OK;
}

int ct_plan_check(const ct_geom *g, const double *angles, int64_t *steps) {
  return ct_plan_check_ex(g, angles, nullptr, steps);
}

int ct_plan_check_ex(const ct_geom *g, const double *angles, const ct_plan_opts *opts,
                     int64_t *steps) {
  clear_error();
  if (!g) {
    set_error("ct_plan_check: null argument");
    return CT_E_INVALID;
  }
  CT_TRY(check_geom(g, angles));
  ct_plan_opts opt;
  CT_TRY(check_opts(opts, &opt));
  return check_plan(g, angles, opt, steps);
}

int ct_objective(const ct_plan *pc, const ct_problem *prob, const float *u, double out[3],
                 ct_stream s) {
  clear_error();
  if (!pc || !prob || !prob->sino || !u || !out) {
    set_error("ct_objective: null argument");
    return CT_E_INVALID;
  }
  ct_plan *p = const_cast<ct_plan *>(pc);
  CT_TRY(plan_scratch(p));
  hipStream_t st = S(s);
  CT_TRY(launch_radon_fwd(p, u, p->d_scratch_sino, st));
  double *d = p->d_red + reduction_partials_needed();
  CT_TRY(launch_objective(p->g.n_angles, p->g.n_bins, p->d_scratch_sino, prob->sino, prob->bound,
                          prob->bound_scalar, prob->mask, p->g.n, (float)(1.0 / p->g.h), u,
                          p->d_red, reduction_partials_needed(), d, st));
  double h[3];
  CT_TRY_HIP(hipMemcpyAsync(h, d, sizeof(double) * 3, hipMemcpyDeviceToHost, st));
  CT_TRY_HIP(hipStreamSynchronize(st));
  out[0] = h[0];
  out[1] = prob->lambda * h[2];
  out[2] = h[1];
  return CT_OK;
}

int ct_plan_destroy(ct_plan *p) {
  clear_error();
  if (!p) return CT_OK;
  free_plan(p);
  delete p;
  return CT_OK;
}

int ct_radon_fwd(const ct_plan *p, const float *img, float *sino, ct_stream s) {
  clear_error();
  if (!p || !img || !sino) {
    set_error("ct_radon_fwd: null argument");
    return CT_E_INVALID;
  }
  return launch_radon_fwd(p, img, sino, S(s));
}

int ct_d0_estimate(const ct_plan *p, const float *u_rec, float threshold, int32_t radius,
                   float kappa, float *chi, float *proj, uint32_t *mask, const float *u0,
                   float c0, float *bound, ct_stream s) {
  clear_error();
  if (!p || !u_rec || !chi || !proj || !mask || ((u0 == nullptr) != (bound == nullptr))) {
    set_error("ct_d0_estimate: null argument (u0 and bound go together)");
    return CT_E_INVALID;
  }
  if (radius < 0 || radius > kDilMaxRadius || !(kappa >= 0.0f) || !std::isfinite(threshold)) {
    set_error("ct_d0_estimate: radius must be in [0, 16], kappa >= 0, threshold finite");
    return CT_E_INVALID;
  }
  return launch_d0_estimate(p, u_rec, threshold, radius, kappa, chi, proj, mask, u0, c0, bound,
                            S(s));
}

int ct_radon_adj(const ct_plan *p, const float *sino, float *img, ct_stream s) {
  clear_error();
  if (!p || !img || !sino) {
    set_error("ct_radon_adj: null argument");
    return CT_E_INVALID;
  }
  return launch_radon_adj(p, sino, nullptr, 1.0f, 0.0f, img, S(s));
}

int ct_grad(int32_t n, double h, const float *u, float *p, ct_stream s) {
  clear_error();
  if (n < 1 || !(h > 0) || !u || !p) {
    set_error("ct_grad: invalid argument");
    return CT_E_INVALID;
  }
  return launch_grad(n, (float)(1.0 / h), u, p, S(s));
}

int ct_div(int32_t n, double h, const float *p, float *d, ct_stream s) {
  clear_error();
  if (n < 2 || !(h > 0) || !p || !d) {
    set_error("ct_div: invalid argument");
    return CT_E_INVALID;
  }
  return launch_div(n, (float)(1.0 / h), p, d, S(s));
}

int ct_precond_create(int32_t n, double sigma, double tau, double c, double eps,
                      ct_precond **out) {
  clear_error();
  if (!out || !(sigma > 0) || !(tau > 0) || !(c > 0) || !(eps > 0)) {
    set_error("ct_precond_create: need sigma, tau, c, eps > 0");
    return CT_E_INVALID;
  }
  *out = nullptr;
  if (!fft_size_ok(n)) {
    set_error("ct_precond_create: n must be even, 2^a 3^b and <= 4096");
    return CT_E_UNSUPPORTED;
  }
  ct_precond *pc = new (std::nothrow) ct_precond();
  if (!pc) return CT_E_DEVICE;
  int rc = precond_init(pc, n, sigma, tau, c, eps);
  if (rc != CT_OK) {
    precond_free(pc);
    delete pc;
    return rc;
  }
  *out = pc;
  return CT_OK;
}

int ct_precond_apply(const ct_precond *m, const float *y, float *x, ct_stream s) {
  clear_error();
  if (!m || !y || !x) {
    set_error("ct_precond_apply: null argument");
    return CT_E_INVALID;
  }
  return launch_apply_mult(m, m->d_mult, y, nullptr, x, S(s));
}

int ct_precond_destroy(ct_precond *m) {
  clear_error();
  if (!m) return CT_OK;
  precond_free(m);
  delete m;
  return CT_OK;
}

int ct_prox_sino(int32_t n_angles, int32_t n_bins, const float *q, double step, const float *u0,
                 const float *bound, const uint32_t *mask, float *y, ct_stream s) {
  clear_error();
  if (n_angles < 1 || n_bins < 1 || !q || !u0 || !y || !(step > 0) || (mask && !bound)) {
    set_error("ct_prox_sino: invalid argument");
    return CT_E_INVALID;
  }
  return launch_prox_sino(n_angles, n_bins, q, (float)step, u0, bound, mask, y, S(s));
}

int ct_tv_project(int32_t n, const float *q, double radius, float *w, ct_stream s) {
  clear_error();
  if (n < 1 || !q || !w || !(radius >= 0)) {
    set_error("ct_tv_project: invalid argument");
    return CT_E_INVALID;
  }
  return launch_tv_project(n, q, (float)radius, w, S(s));
}

int ct_power_norm(const ct_plan *pc, int32_t iters, const float *x0, double *out, ct_stream s) {
  clear_error();
  if (!pc || !out || iters < 1) {
    set_error("ct_power_norm: invalid argument");
    return CT_E_INVALID;
  }
  ct_plan *p = const_cast<ct_plan *>(pc);
  CT_TRY(plan_scratch(p));
  const int n = p->g.n;
  const size_t nn = (size_t)n * n;
  float *x = p->d_scratch_img, *y = p->d_scratch_img + nn;
  hipStream_t st = S(s);
  if (x0) {
    CT_TRY_HIP(hipMemcpyAsync(x, x0, sizeof(float) * nn, hipMemcpyDeviceToDevice, st));
  } else {
    auto h0 = default_start(n);
    CT_TRY_HIP(hipMemcpyAsync(x, h0.data(), sizeof(float) * nn, hipMemcpyHostToDevice, st));
    CT_TRY_HIP(hipStreamSynchronize(st));
  }
  double *d_norm = p->d_red + reduction_partials_needed();
  double lam = 0;
  auto op = [&](float *xin, float *yout) -> int {
    CT_TRY(launch_radon_fwd(p, xin, p->d_scratch_sino, st));
    return launch_radon_adj(p, p->d_scratch_sino, nullptr, 1.0f, 0.0f, yout, st);
  };
  CT_TRY(power_iterate(n, iters, x, y, p->d_red, p->red_cap, d_norm, op, st, &lam));
  *out = std::sqrt(lam);
  return CT_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Solver: nb >= 1 problems of one geometry advanced together.  Every state
// array holds the nb problems one after the other ([nb][n][n], [nb][N][M],
// ...); each kernel of an iteration covers all of them in one launch.

static int solver_alloc(ct_solver *sv) {
  const size_t nb = sv->nb;
  const size_t nn = (size_t)sv->n * sv->n * nb, NM = (size_t)sv->N * sv->M * nb;
  CT_TRY_HIP(hipMalloc(&sv->u, sizeof(float) * nn));
  CT_TRY_HIP(hipMalloc(&sv->u_next, sizeof(float) * nn));
  CT_TRY_HIP(hipMalloc(&sv->utmp, sizeof(float) * nn));
  CT_TRY_HIP(hipMalloc(&sv->vb2, sizeof(float) * nn * 2));
  CT_TRY_HIP(hipMalloc(&sv->s2, sizeof(float) * nn * 2));
  CT_TRY_HIP(hipMalloc(&sv->w, sizeof(float) * nn * 2));
  CT_TRY_HIP(hipMalloc(&sv->vb1, sizeof(float) * NM));
  CT_TRY_HIP(hipMalloc(&sv->s1, sizeof(float) * NM));
  CT_TRY_HIP(hipMalloc(&sv->target, sizeof(float) * NM));
  // one sinogram: the set-up's projections of a single image
  CT_TRY_HIP(hipMalloc(&sv->rraw, sizeof(float) * (size_t)sv->N * sv->M));
  CT_TRY_HIP(hipMalloc(&sv->y1, sizeof(float) * NM));
  CT_TRY_HIP(hipMalloc(&sv->r, sizeof(float) * NM));
  const size_t MW = (size_t)(sv->M + 31) / 32;
  CT_TRY_HIP(hipMalloc(&sv->mask, sizeof(uint32_t) * sv->N * MW * nb));
  CT_TRY_HIP(hipMalloc(&sv->spec, sizeof(float2) * (size_t)(sv->n / 2 + 1) * sv->n * nb));
  sv->red_cap = reduction_partials_needed() + 16;
  CT_TRY_HIP(hipMalloc(&sv->d_red, sizeof(double) * sv->red_cap));
  CT_TRY_HIP(hipMalloc(&sv->d_out, sizeof(double) * 16));
  return CT_OK;
}

// Partial images of the sliced backprojection: nb * S images.
static int solver_set_slices(ct_solver *sv, int S) {
  const size_t need = (S > 1) ? (size_t)S * sv->nb * sv->n * sv->n : 0;
  if (need > sv->bp_cap) {
    (void)hipFree(sv->bp_part);
    sv->bp_part = nullptr;
    sv->bp_cap = 0;
    CT_TRY_HIP(hipMalloc(&sv->bp_part, sizeof(float) * need));
    sv->bp_cap = need;
  }
  sv->bp_S = S;
  return CT_OK;
}

// R_h of the iteration with `walk` angles per walk: the plan's own tables
// when they have that walk, else forward tables of the solver's own (a mode
// that falls back to the plan's walk uses the plan's tables).
static int solver_set_walk(ct_solver *sv, int walk) {
  ct_plan *p = sv->plan;
  if (walk != p->slots && sv->fwd_alt && sv->fwd_alt_walk == walk) {
    sv->fwd = sv->fwd_alt;
    return CT_OK;
  }
  if (sv->fwd_alt) {
    free_plan(sv->fwd_alt);
    delete sv->fwd_alt;
    sv->fwd_alt = nullptr;
    sv->fwd_alt_walk = 0;
  }
  sv->fwd = p;
  if (walk == p->slots) return CT_OK;
  ct_plan *a = new (std::nothrow) ct_plan();
  if (!a) return CT_E_DEVICE;
  const int rc = build_fwd_plan(p, walk, a);
  if (rc != CT_OK || a->slots == p->slots) {
    free_plan(a);
    delete a;
    return rc;
  }
  sv->fwd_alt = a;
  sv->fwd_alt_walk = walk;
  sv->fwd = a;
  return CT_OK;
}

static int solver_zero_state(ct_solver *sv, hipStream_t s) {
  const size_t nn = (size_t)sv->n * sv->n * sv->nb, NM = (size_t)sv->N * sv->M * sv->nb;
  CT_TRY_HIP(hipMemsetAsync(sv->u, 0, sizeof(float) * nn, s));
  CT_TRY_HIP(hipMemsetAsync(sv->u_next, 0, sizeof(float) * nn, s));
  CT_TRY_HIP(hipMemsetAsync(sv->vb2, 0, sizeof(float) * nn * 2, s));
  CT_TRY_HIP(hipMemsetAsync(sv->s2, 0, sizeof(float) * nn * 2, s));
  CT_TRY_HIP(hipMemsetAsync(sv->vb1, 0, sizeof(float) * NM, s));
  CT_TRY_HIP(hipMemsetAsync(sv->s1, 0, sizeof(float) * NM, s));
  if (sv->ubar) CT_TRY_HIP(hipMemsetAsync(sv->ubar, 0, sizeof(float) * nn, s));
  if (sv->ucp) CT_TRY_HIP(hipMemsetAsync(sv->ucp, 0, sizeof(float) * nn, s));
  // PDRQS2 caches the residual b - A u, which is b at u = 0
  if (sv->method == CT_METHOD_PDRQS2)
    CT_TRY_HIP(hipMemcpyAsync(sv->s1, sv->target, sizeof(float) * NM, hipMemcpyDeviceToDevice, s));
  // PDRQS3 caches D (vb1 + sigma (A u - g)), -sigma b / (1 + sigma) off D0 at u = 0
  if (sv->method == CT_METHOD_PDRQS3) {
    const SinoEpi ep{(float)(1.0 / sv->beta), (float)sv->sigma, sv->target, sv->mask, sv->vb1,
                     sv->s1, nullptr, nullptr, 8};
    CT_TRY(launch_radon_fwd(sv->fwd, sv->u, nullptr, s, &ep, sv->nb));
  }
  sv->iters = 0;
  sv->have_dual = false;
  return CT_OK;
}

// One PDRQS1 iteration (§4.4) of all nb problems from the cached
// s1 = vb1 + sigma A u, s2 = vb2 + sigma tau nabla u; mode 2 keeps y1, w and
// A u for the record.  With ev (5 events) the phase boundaries are recorded.
// Algorithm CP (§3.4) on the normalized problem: dual steps at the
// extrapolated iterate ucp, then the primal step with its extrapolation.
// Steps sigma = tau = 0.99 / sqrt(1 + 8/h^2) (sigma tau ||K||^2 < 1 with
// ||A|| = 1 after the normalization and ||nabla_h||^2 < 8/h^2).
static int cp_iter(ct_solver *sv, hipStream_t st) {
  ct_plan *p = sv->plan;
  const double h = p->g.h;
  const float step = (float)(0.99 / std::sqrt(1.0 + 8.0 / (h * h)));
  const int nb = sv->nb;
  const SinoEpi ep{(float)(1.0 / sv->beta), step, sv->target, sv->mask, sv->vb1, nullptr,
                   nullptr, nullptr, 4};
  CT_TRY(launch_radon_fwd(sv->fwd, sv->ucp, nullptr, st, &ep, nb));
  CT_TRY(launch_tv_update(sv->n, (float)(1.0 / h), sv->ucp, step, (float)sv->lam_t, sv->vb2,
                          nullptr, nullptr, 4, st, nb));
  CT_TRY(launch_radon_adj(p, sv->vb1, sv->vb2, (float)(-step / sv->beta), step, sv->u_next, st,
                          nb, sv->bp_part, sv->bp_S, sv->bp_kern, sv->u, nullptr, sv->ucp));
  std::swap(sv->u, sv->u_next);
  sv->iters += 1;
  return CT_OK;
}

// One ADMM iteration (§4.6) on the normalized unconstrained problem (nb = 1):
// the PCG u-step on H u = A^*(z_w - eta_w) - tau^2 div(z_v - eta_v),
// H = A^* A - tau^2 div nabla, from the current u; then the z-step and the
// multiplier update, fused into the epilogues of R_h u and nabla_h u.
static int admm_iter(ct_solver *sv, hipStream_t st) {
  ct_plan *p = sv->plan;
  const int64_t nn = (int64_t)sv->n * sv->n;
  const float inv_h = (float)(1.0 / p->g.h);
  const float t2 = (float)(sv->tau * sv->tau);
  const float inv_b = (float)(1.0 / sv->beta), inv_b2 = (float)(1.0 / (sv->beta * sv->beta));
  double *sc = sv->d_cg, *part = sv->d_cg + 4;
  // r = rhs - H u = A^*((z_w - eta_w) - A u) - tau^2 div((z_v - eta_v) - nabla u)
  CT_TRY(launch_radon_adj(p, sv->s1, sv->s2, inv_b, -t2, sv->cg_r, st, 1, sv->bp_part,
                          sv->bp_S, sv->bp_kern));
  CT_TRY(launch_apply_mult(&sv->pc, sv->pc.d_mult, sv->cg_r, nullptr, sv->cg_z, st));
  CT_TRY(launch_dot(sv->cg_r, sv->cg_z, nn, part, sc + 0, st));
  CT_TRY(launch_cg_dir(nn, nullptr, nullptr, sv->cg_z, sv->cg_p, st));
  int cur = 0;
  for (int k = 0; k < sv->admm_cg; ++k) {
    // Hp = A^*(A p) - tau^2 div(nabla p)
    CT_TRY(launch_radon_fwd(sv->fwd, sv->cg_p, sv->r, st));
    CT_TRY(launch_grad(sv->n, inv_h, sv->cg_p, sv->w, st));
    CT_TRY(launch_radon_adj(p, sv->r, sv->w, inv_b2, -t2, sv->cg_Hp, st, 1, sv->bp_part,
                            sv->bp_S, sv->bp_kern));
    CT_TRY(launch_dot(sv->cg_p, sv->cg_Hp, nn, part, sc + 2, st));
    CT_TRY(launch_cg_update(nn, sc + cur, sc + 2, sv->cg_p, sv->cg_Hp, sv->u, sv->cg_r, st));
    if (k + 1 < sv->admm_cg) {  // the direction after the last step is not used
      CT_TRY(launch_apply_mult(&sv->pc, sv->pc.d_mult, sv->cg_r, nullptr, sv->cg_z, st));
      CT_TRY(launch_dot(sv->cg_r, sv->cg_z, nn, part, sc + (1 - cur), st));
      CT_TRY(launch_cg_dir(nn, sc + (1 - cur), sc + cur, sv->cg_z, sv->cg_p, st));
      cur = 1 - cur;
    }
  }
  // z-step and eta update from A u and nabla u (mu travels in the sigma field)
  const SinoEpi ep{inv_b, (float)sv->admm_mu, sv->target, nullptr, sv->vb1, sv->s1, nullptr,
                   nullptr, 6};
  CT_TRY(launch_radon_fwd(sv->fwd, sv->u, nullptr, st, &ep));
  CT_TRY(launch_tv_update(sv->n, inv_h, sv->u, 0.f,
                          (float)(sv->lam_t / (sv->admm_mu * sv->tau * sv->tau)), sv->vb2,
                          sv->s2, nullptr, 5, st));
  sv->iters += 1;
  return CT_OK;
}

static int solver_iter(ct_solver *sv, int mode, hipStream_t st, hipEvent_t *ev = nullptr,
                       float *q1out = nullptr, float *q2out = nullptr) {
  if (sv->method == CT_METHOD_CP) return cp_iter(sv, st);
  if (sv->method == CT_METHOD_ADMM) return admm_iter(sv, st);
  ct_plan *p = sv->plan;
  const float sig = (float)sv->sigma, tau = (float)sv->tau;
  const float inv_h = (float)(1.0 / p->g.h);
  const int nb = sv->nb;
  if (sv->method == CT_METHOD_PDRQS2) {
    // §4.2: u_tmp = sigma A^*(b - A u) + sigma tau div(vb2 + sigma tau nabla u)
    BpDeferred def{};
    CT_TRY(launch_radon_adj(p, sv->s1, sv->s2, (float)(sv->sigma / sv->beta),
                            (float)(sv->sigma * sv->tau), sv->utmp, st, nb, sv->bp_part,
                            sv->bp_S, sv->bp_kern, nullptr, nullptr, nullptr,
                            sv->defer_combine ? &def : nullptr));
    CT_TRY(launch_apply_mult(&sv->pc, sv->pc.d_mult, sv->utmp, sv->u, sv->u_next, st, nb,
                             sv->spec, def.S > 1 ? &def : nullptr));
    const SinoEpi ep{(float)(1.0 / sv->beta), sig, sv->target, nullptr, nullptr, sv->s1,
                     nullptr, nullptr, 5};
    CT_TRY(launch_radon_fwd(sv->fwd, sv->u_next, nullptr, st, &ep, nb));
    CT_TRY(launch_tv_update(sv->n, inv_h, sv->u_next, sig * tau, (float)(sv->lam_t / sv->tau),
                            sv->vb2, sv->s2, sv->w, mode == 2 ? 2 : 0, st, nb));
    std::swap(sv->u, sv->u_next);
    sv->iters += 1;
    return CT_OK;
  }
  if (ev) CT_TRY_HIP(hipEventRecord(ev[0], st));
  // u_tmp (u >= 0 variant: plus bar u - u); with angle slices and the FFT
  // pair next, the slices' sum and epilogue are formed in the FFT's row pass
  BpDeferred def{};
  const bool rich = sv->method == CT_METHOD_RICHARDSON;
  CT_TRY(launch_radon_adj(p, sv->s1, sv->s2, (float)(-sv->sigma / sv->beta),
                          (float)(sv->sigma * sv->tau), sv->utmp, st, nb, sv->bp_part, sv->bp_S,
                          sv->bp_kern, sv->ubar, sv->ubar ? sv->u : nullptr, nullptr,
                          rich || !sv->defer_combine ? nullptr : &def));
  if (ev) CT_TRY_HIP(hipEventRecord(ev[1], st));
  if (rich)
    CT_TRY(launch_axpy((int64_t)sv->n * sv->n * nb, sv->u, (float)(1.0 / sv->rich_m), sv->utmp,
                       sv->u_next, st));
  else
    CT_TRY(launch_apply_mult(&sv->pc, sv->pc.d_mult, sv->utmp, sv->u, sv->u_next, st, nb,
                             sv->spec, def.S > 1 ? &def : nullptr));
  if (ev) CT_TRY_HIP(hipEventRecord(ev[2], st));
  // R_h u_new with the sinogram-side update fused into its output stage
  SinoEpi ep{(float)(1.0 / sv->beta), sig, sv->target, sv->mask, sv->vb1, sv->s1,
             sv->y1, sv->r, sv->method == CT_METHOD_PDRQS3 ? 7 : mode};
  ep.q1 = q1out;
  ep.fit = sv->fit;
  ep.aux = sv->fit_aux;
  // the gradient-side update reads u_new only: it runs in the same launch
  // (extra workgroups), also when the phases are timed one by one
  TvArgs tv;
  tv.n = sv->n;
  tv.inv_h = inv_h;
  tv.u = sv->u_next;
  tv.st = sig * tau;
  tv.radius = (float)(sv->lam_t / sv->tau);
  tv.vb2 = sv->vb2;
  tv.s2 = sv->s2;
  tv.wout = sv->w;
  tv.mode = mode;
  tv.q2out = q2out;
  tv.ubar = sv->ubar;
  tv.blocks = sv->fuse_tv ? sv->tv_blocks : 0;
  bool fused = false;
  CT_TRY(launch_radon_fwd(sv->fwd, sv->u_next, nullptr, st, &ep, nb, &tv, &fused));
  if (ev) CT_TRY_HIP(hipEventRecord(ev[3], st));
  if (!fused)
    CT_TRY(launch_tv_update(sv->n, inv_h, sv->u_next, sig * tau, (float)(sv->lam_t / sv->tau),
                            sv->vb2, sv->s2, sv->w, mode, st, nb, q2out, sv->ubar));
  if (ev) CT_TRY_HIP(hipEventRecord(ev[4], st));
  std::swap(sv->u, sv->u_next);
  sv->iters += 1;
  return CT_OK;
}

// Tuning results kept in a JSON file (ct_params.tune_cache): one entry per
// line, {"key": "...", "bp_kernel": k, "bp_slices": S, "tv_blocks": b,
// "fwd_walk": w}, between a header line and a closing line.  The key names
// the device (its architecture and compute-unit count), the library version,
// the geometry, the plan's own walk, the batch size and the method class.
struct TuneChoice {
  int kern = 4, S = 1, tv_blocks = 256, walk = 2;
};

static std::string tune_key(const ct_solver *sv, bool with_fft, bool tvf) {
  const ct_plan *p = sv->plan;
  hipDeviceProp_t prop;
  std::string arch = "unknown";
  int cus = 0;
  if (hipGetDeviceProperties(&prop, p->device) == hipSuccess) {
    arch = prop.gcnArchName;
    cus = prop.multiProcessorCount;
  }
  for (char &c : arch)
    if (c == '"' || c == '\\' || c == '\n') c = '_';
  char buf[512];
  std::snprintf(buf, sizeof(buf),
                "%s/cu%d/v%d/n%d/N%d/M%d/h%.17g/ds%.17g/ang%016llx/walk%d/nb%d/fft%d/tvf%d",
                arch.c_str(), cus, ct_version(), p->g.n, p->g.n_angles, p->g.n_bins, p->g.h,
                p->g.ds, (unsigned long long)p->angles_hash, p->slots, sv->nb, with_fft ? 1 : 0,
                tvf ? 1 : 0);
  return buf;
}

static bool tune_line_parse(const std::string &line, std::string *key, TuneChoice *c) {
  const std::string kk = "{\"key\": \"";
  if (line.compare(0, kk.size(), kk) != 0) return false;
  const size_t q = line.find('"', kk.size());
  if (q == std::string::npos) return false;
  *key = line.substr(kk.size(), q - kk.size());
  auto field = [&](const char *name, int *v) {
    const std::string f = std::string("\"") + name + "\": ";
    const size_t at = line.find(f, q);
    if (at == std::string::npos) return false;
    char *end = nullptr;
    const long x = std::strtol(line.c_str() + at + f.size(), &end, 10);
    if (end == line.c_str() + at + f.size()) return false;
    *v = (int)x;
    return true;
  };
  return field("bp_kernel", &c->kern) && field("bp_slices", &c->S) &&
         field("tv_blocks", &c->tv_blocks) && field("fwd_walk", &c->walk);
}

static std::vector<std::pair<std::string, TuneChoice>> tune_file_read(const char *path) {
  std::vector<std::pair<std::string, TuneChoice>> out;
  FILE *f = std::fopen(path, "r");
  if (!f) return out;
  std::string line;
  int ch;
  while (true) {
    line.clear();
    while ((ch = std::fgetc(f)) != EOF && ch != '\n') line.push_back((char)ch);
    std::string key;
    TuneChoice c;
    if (tune_line_parse(line, &key, &c)) out.emplace_back(key, c);
    if (ch == EOF) break;
  }
  std::fclose(f);
  return out;
}

// Adds (or replaces) one entry; the file is rewritten whole through a
// temporary file and a rename, so that a reader never sees half a file.
static bool tune_file_store(const char *path, const std::string &key, const TuneChoice &c) {
  auto all = tune_file_read(path);
  bool found = false;
  for (auto &e : all)
    if (e.first == key) {
      e.second = c;
      found = true;
    }
  if (!found) all.emplace_back(key, c);
  const std::string tmp = std::string(path) + ".tmp" + std::to_string((long)getpid());
  FILE *f = std::fopen(tmp.c_str(), "w");
  if (!f) return false;
  std::fprintf(f, "{\"format\": \"ctpd-tune\", \"entries\": [\n");
  for (size_t q = 0; q < all.size(); ++q)
    std::fprintf(f,
                 "{\"key\": \"%s\", \"bp_kernel\": %d, \"bp_slices\": %d, \"tv_blocks\": %d, "
                 "\"fwd_walk\": %d}%s\n",
                 all[q].first.c_str(), all[q].second.kern, all[q].second.S,
                 all[q].second.tv_blocks, all[q].second.walk, q + 1 < all.size() ? "," : "");
  std::fprintf(f, "]}\n");
  const bool ok = std::fclose(f) == 0;
  if (!ok || std::rename(tmp.c_str(), path) != 0) {
    (void)std::remove(tmp.c_str());
    return false;
  }
  return true;
}

// A stored choice is used only if it is one this solver could make.
static bool tune_choice_valid(const ct_solver *sv, const TuneChoice &c) {
  const bool kern_ok = c.kern == 0 || ((c.kern == 4 || c.kern == 8) && sv->plan->n_bpp > 0);
  return kern_ok && c.S >= 1 && c.S <= kMaxSlices && c.tv_blocks >= 0 && c.tv_blocks <= 4096 &&
         (c.walk == 1 || c.walk == 2 || c.walk == 4);
}

// The launch choices of the iteration: the angles per walk of R_h, the
// backprojector (mirror pairs on 32 x 32 or 32 x 64 tiles, or one angle at a
// time), its number of angle slices, and the workgroups that run the
// gradient-side update inside R_h's launch (0: a launch of its own).  What
// the params (or a plan created with a fixed walk) fix is kept; with
// CT_OPT_NO_TUNE the rest are the plan's defaults.  Otherwise, when nothing
// is fixed, a choice recorded for this plan and batch size (an earlier
// solver) or in the tune cache file is reused; else the candidates are timed
// on the solver's own data (the caches s1, s2 of the zero state): R_h of the
// zero image with each walk, together with the gradient-side update as the
// iteration runs it; the backprojection together with the pass that sums its
// slices (the FFT pair or the combine); then R_h's launch with each number of
// extra workgroups.
static int solver_tune(ct_solver *sv, const ct_params *prm, hipStream_t st) {
  ct_plan *p = sv->plan;
  const int N = sv->N;
  const bool with_fft = sv->defer_combine &&
                        (sv->method == CT_METHOD_PDRQS1 || sv->method == CT_METHOD_PDRQS2 ||
                         sv->method == CT_METHOD_PDRQS3);
  // the gradient-side update joins R_h's launch in the PDRQS1-type
  // iterations when R_h walks several angles at a time (launch_radon_fwd)
  const bool tvf = sv->fuse_tv &&
                   (sv->method == CT_METHOD_PDRQS1 || sv->method == CT_METHOD_RICHARDSON ||
                    sv->method == CT_METHOD_PDRQS3);
  const bool kern_fixed = prm->bp_kernel != CT_BP_AUTO;
  const bool S_fixed = prm->bp_slices > 0;
  const bool walk_fixed = prm->fwd_walk != 0 || p->walk_opt != 0;
  TuneChoice ch;
  ch.kern = kern_fixed ? (p->n_bpp > 0 ? prm->bp_kernel : 0) : p->bp_kern0;
  ch.S = S_fixed ? prm->bp_slices : p->bp_slices;
  ch.tv_blocks = prm->tv_blocks > 0 ? prm->tv_blocks : std::min(sv->n, 256);
  ch.walk = prm->fwd_walk != 0 ? prm->fwd_walk : p->slots;
  const bool tv_fixed = prm->tv_blocks > 0 || !tvf || (walk_fixed && ch.walk == 1);
  sv->tune_source = 0;
  sv->tune_timed = 0;
  sv->tune_saved = 0;
  auto apply = [&]() -> int {
    sv->bp_kern = ch.kern;
    sv->tv_blocks = ch.tv_blocks;
    CT_TRY(solver_set_walk(sv, ch.walk));
    return solver_set_slices(sv, ch.S);
  };
  const bool all_free = !kern_fixed && !S_fixed && prm->tv_blocks == 0 && !walk_fixed;
  if ((prm->options & CT_OPT_NO_TUNE) || (kern_fixed && S_fixed && tv_fixed && walk_fixed))
    return apply();
  std::string key;
  if (all_free) {
    for (const auto &t : p->tune_cache)
      if (t.nb == sv->nb && t.fft == (int)with_fft && t.tvf == (int)tvf) {
        ch = TuneChoice{t.kern, t.S, t.tv_blocks, t.walk};
        sv->tune_source = 2;
        return apply();
      }
    if (prm->tune_cache) {
      key = tune_key(sv, with_fft, tvf);
      for (const auto &e : tune_file_read(prm->tune_cache))
        if (e.first == key && tune_choice_valid(sv, e.second)) {
          ch = e.second;
          sv->tune_source = 3;
          p->tune_cache.push_back(ct_plan::TuneEntry{sv->nb, (int)with_fft, (int)tvf, ch.kern,
                                                     ch.S, ch.tv_blocks, ch.walk});
          return apply();
        }
    }
  }
  struct Cand {
    int kern;  // mirror pairs with 4 or 8 pixels per thread; 0: one angle at a time
    int S;
  };
  std::vector<Cand> cands;
  // mirror pairs on small tiles are tried for one problem only (a batch
  // fills the device with larger tiles' workgroups)
  for (int kern : {4, 8, 0}) {
    if (kern_fixed) {
      if (kern != ch.kern) continue;
    } else {
      if (kern != 0 && p->n_bpp == 0) continue;
      if (kern == 4 && sv->nb != 1) continue;
    }
    if (S_fixed) {
      cands.push_back(Cand{kern, ch.S});
      continue;
    }
    // staged chunks of the backprojection's angles (mirror pairs when paired)
    const int items = kern ? p->n_bpp / kBpPairChunk : N / kBpChunk;
    for (int S : {1, 2, 4, 8, kMaxSlices})
      if (S == 1 || items / S >= 2) cands.push_back(Cand{kern, S});
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  CT_TRY_HIP(hipEventCreate(&e0));
  std::unique_ptr<std::remove_pointer<hipEvent_t>::type, hipError_t (*)(hipEvent_t)> g0(
      e0, hipEventDestroy);
  CT_TRY_HIP(hipEventCreate(&e1));
  std::unique_ptr<std::remove_pointer<hipEvent_t>::type, hipError_t (*)(hipEvent_t)> g1(
      e1, hipEventDestroy);
  auto time_it = [&](auto &&run, float *ms) -> int {
    CT_TRY(run());  // warm-up
    CT_TRY_HIP(hipEventRecord(e0, st));
    for (int r = 0; r < 4; ++r) CT_TRY(run());
    CT_TRY_HIP(hipEventRecord(e1, st));
    CT_TRY_HIP(hipEventSynchronize(e1));
    CT_TRY_HIP(hipEventElapsedTime(ms, e0, e1));
    sv->tune_timed += 1;
    return CT_OK;
  };
  // The index of the fastest of count candidates: each is timed once per
  // round (prepare(c), then run(c) through time_it), rounds interleaved so
  // that clock and thermal drift reach every candidate alike, and its best
  // round kept; after the first round only candidates within 15 % of the
  // best are timed again.  Ties go to the earlier candidate.
  constexpr int kTuneRounds = 3;
  auto pick = [&](int count, auto &&prepare, auto &&run, int *best) -> int {
    std::vector<float> t(count, 0.f);
    for (int r = 0; r < kTuneRounds; ++r) {
      const float cut = r == 0 ? 0.f : 1.15f * *std::min_element(t.begin(), t.end());
      for (int c = 0; c < count; ++c) {
        if (r > 0 && t[c] > cut) continue;
        CT_TRY(prepare(c));
        float ms = 0.f;
        CT_TRY(time_it([&]() { return run(c); }, &ms));
        if (r == 0 || ms < t[c]) t[c] = ms;
      }
    }
    *best = 0;
    for (int c = 1; c < count; ++c)
      if (t[c] < t[*best]) *best = c;
    return CT_OK;
  };
  // R_h of the zero image with the gradient-side update of the zero state
  // (u_new = 0 leaves vb2 = s2 = 0, and bar u = 0): the state is unchanged.
  // The raw projections of the nb problems go to y1 ([nb][N][M]; it holds
  // nothing before the first iteration).  blocks: the update's workgroups in
  // R_h's launch (0: a launch of its own); R_h alone where the method does
  // not run the update next to it.
  const size_t nn = (size_t)sv->n * sv->n * sv->nb;
  CT_TRY_HIP(hipMemsetAsync(sv->u_next, 0, sizeof(float) * nn, st));
  const float sig = (float)sv->sigma, tau = (float)sv->tau;
  const float inv_h = (float)(1.0 / p->g.h);
  auto time_fwd_run = [&](const ct_plan *fp, int blocks) -> int {
    TvArgs tv;
    tv.n = sv->n;
    tv.inv_h = inv_h;
    tv.u = sv->u_next;
    tv.st = sig * tau;
    tv.radius = (float)(sv->lam_t / sv->tau);
    tv.vb2 = sv->vb2;
    tv.s2 = sv->s2;
    tv.wout = sv->w;
    tv.mode = 0;
    tv.ubar = sv->ubar;
    tv.blocks = blocks;
    bool fused = false;
    CT_TRY(launch_radon_fwd(fp, sv->u_next, sv->y1, st, nullptr, sv->nb, tvf ? &tv : nullptr,
                            &fused));
    if (tvf && !fused)
      CT_TRY(launch_tv_update(sv->n, inv_h, sv->u_next, sig * tau, tv.radius, sv->vb2, sv->s2,
                              sv->w, 0, st, sv->nb, nullptr, sv->ubar));
    return CT_OK;
  };
  if (!walk_fixed) {
    // 4, 2 and 1 angles per walk, each with its forward tables as built (a
    // mode that falls back to another is timed as that other one)
    struct PlanFree {
      void operator()(ct_plan *a) const {
        free_plan(a);
        delete a;
      }
    };
    std::vector<int> walks;
    std::vector<std::unique_ptr<ct_plan, PlanFree>> tabs;  // null: the plan's own
    for (int w : {4, 2, 1}) {
      std::unique_ptr<ct_plan, PlanFree> own;
      if (w != p->slots) {
        own.reset(new (std::nothrow) ct_plan());
        if (!own) return CT_E_DEVICE;
        if (build_fwd_plan(p, w, own.get()) != CT_OK || own->slots != w) {
          clear_error();
          continue;
        }
      }
      walks.push_back(w);
      tabs.push_back(std::move(own));
    }
    int bi = 0;
    CT_TRY(pick(
        (int)walks.size(), [](int) { return CT_OK; },
        [&](int c) {
          return time_fwd_run(tabs[c] ? tabs[c].get() : p, walks[c] >= 2 ? ch.tv_blocks : 0);
        },
        &bi));
    ch.walk = walks[bi];
    if (tabs[bi]) {
      if (sv->fwd_alt) {
        free_plan(sv->fwd_alt);
        delete sv->fwd_alt;
      }
      sv->fwd_alt = tabs[bi].release();
      sv->fwd_alt_walk = ch.walk;
    }
  }
  CT_TRY(solver_set_walk(sv, ch.walk));
  if (cands.size() > 1) {
    // what the iteration runs: with the FFT pair next, R_h^* with its slice
    // sum deferred into the row pass and the pair itself; else R_h^* and the
    // slice combine
    auto run = [&](int c) -> int {
      const int kern = cands[c].kern;
      if (!with_fft)
        return launch_radon_adj(p, sv->s1, sv->s2, 1.0f, 0.0f, sv->utmp, st, sv->nb,
                                sv->bp_part, sv->bp_S, kern);
      BpDeferred def{};
      CT_TRY(launch_radon_adj(p, sv->s1, sv->s2, 1.0f, 0.0f, sv->utmp, st, sv->nb, sv->bp_part,
                              sv->bp_S, kern, nullptr, nullptr, nullptr, &def));
      return launch_apply_mult(&sv->pc, sv->pc.d_mult, sv->utmp, sv->u, sv->u_next, st, sv->nb,
                               sv->spec, def.S > 1 ? &def : nullptr);
    };
    int bi = 0;
    CT_TRY(pick(
        (int)cands.size(), [&](int c) { return solver_set_slices(sv, cands[c].S); }, run, &bi));
    ch.kern = cands[bi].kern;
    ch.S = cands[bi].S;
  }
  if (!tv_fixed && sv->fwd->slots >= 2) {
    // the backprojection candidates wrote u_next (u + M^{-1} u_tmp, not zero
    // where the zero state's s1 is not): zero again, so that the update
    // leaves the state as it is
    CT_TRY_HIP(hipMemsetAsync(sv->u_next, 0, sizeof(float) * nn, st));
    std::vector<int> blocks;
    for (int b : {64, 128, 256, 512, 1024})
      if (b <= sv->n) blocks.push_back(b);
    if (blocks.empty()) blocks.push_back(sv->n);
    blocks.push_back(0);  // a launch of its own
    int bi = 0;
    CT_TRY(pick(
        (int)blocks.size(), [](int) { return CT_OK; },
        [&](int c) { return time_fwd_run(sv->fwd, blocks[c]); }, &bi));
    ch.tv_blocks = blocks[bi];
  }
  if (!sv->tune_timed) return apply();
  sv->tune_source = 1;
  if (all_free) {
    p->tune_cache.push_back(ct_plan::TuneEntry{sv->nb, (int)with_fft, (int)tvf, ch.kern, ch.S,
                                               ch.tv_blocks, ch.walk});
    if (prm->tune_cache) sv->tune_saved = tune_file_store(prm->tune_cache, key, ch) ? 1 : 0;
  }
  return apply();
}

// Kernel preconditioners for PDRQS1, built from the response of A^* A to a
// unit impulse at pixel (n/2, n/2):
//  * impulse response (§4.3.2): the response centred at the origin and
//    averaged over the eight symmetries of the square, a 2-D convolution
//    kernel k; F(K) = sigma^2 F(k) + (sigma tau)^2 lambda_Delta;
//  * circulant (§4.3.3): on the column-major vectorized image (index
//    m = j + n i, length L = n^2), the response shifted to index 0 and
//    symmetrized, (c_m + c_{L-m}) / 2, the first column of a circulant;
//    F_L(K) = sigma^2 F_L(k) + (sigma tau)^2 (4 - 2 cos(2 pi q/L) - 2 cos(2 pi q/n)),
//    applied by the FFT pair with the twiddle between its passes (pc.twist).
// c = c_safety lambda_max(M_K^{-1} T) by power iteration unless given,
// T = sigma^2 A^* A - (sigma tau)^2 div nabla; multiplier 1 / (c F(K)).
// F(k) comes from the FFT pair itself: with the kernel as the multiplier
// table (unnormalized) and a unit impulse at the origin as input, the pair
// returns the (even, real) transform of the kernel.
static int kernel_precond_setup(ct_solver *sv, const ct_params *prm, bool circ, hipStream_t st) {
  ct_plan *p = sv->plan;
  const int n = sv->n, half = n / 2 + 1;
  const size_t nn = (size_t)n * n;
  const double sig = sv->sigma, st2 = (sv->sigma * sv->tau) * (sv->sigma * sv->tau);
  std::vector<float> img(nn, 0.f);
  img[(size_t)(n / 2) * n + n / 2] = 1.f;
  CT_TRY_HIP(hipMemcpyAsync(sv->u, img.data(), sizeof(float) * nn, hipMemcpyHostToDevice, st));
  CT_TRY(launch_radon_fwd(p, sv->u, sv->rraw, st));
  CT_TRY(launch_radon_adj(p, sv->rraw, nullptr, (float)(1.0 / (sv->beta * sv->beta)), 0.0f,
                          sv->utmp, st, 1, sv->bp_part, sv->bp_S));
  std::vector<float> kt(nn);
  CT_TRY_HIP(hipMemcpyAsync(kt.data(), sv->utmp, sizeof(float) * nn, hipMemcpyDeviceToHost, st));
  CT_TRY_HIP(hipStreamSynchronize(st));
  std::vector<float> tab((size_t)half * n);
  if (!circ) {
    // k(x1, x2) = mean over g of kt(n/2 + g(x)), indices modulo n; as the
    // table m[x1][x2] for x1 in [0, n/2] (k is even, the other half mirrors it)
    auto at = [&](int y, int x) {
      return (double)kt[(size_t)((y + n / 2) % n) * n + (size_t)((x + n / 2) % n)];
    };
    for (int x1 = 0; x1 < half; ++x1)
      for (int x2 = 0; x2 < n; ++x2) {
        const int a = x1, b = x2, na = (n - a) % n, nb2 = (n - b) % n;
        const double v = at(b, a) + at(b, na) + at(nb2, a) + at(nb2, na) + at(a, b) +
                         at(a, nb2) + at(na, b) + at(na, nb2);
        tab[(size_t)x1 * n + x2] = (float)(v / 8.0);
      }
  } else {
    // k_m = (c_m + c_{L-m}) / 2 with c_m = kt at vector index (m + m0) mod L;
    // as the table m[k1][k2] = k_{k1 + n k2}, k1 in [0, n/2] (k is symmetric)
    const int64_t L = (int64_t)n * n, m0 = n / 2 + (int64_t)n * (n / 2);
    auto cvec = [&](int64_t m) {
      const int64_t v = ((m + m0) % L + L) % L;
      const int64_t j = v % n, i = v / n;
      return (double)kt[(size_t)j * n + (size_t)i];
    };
    for (int k1 = 0; k1 < half; ++k1)
      for (int k2 = 0; k2 < n; ++k2) {
        const int64_t m = k1 + (int64_t)n * k2;
        tab[(size_t)k1 * n + k2] = (float)(0.5 * (cvec(m) + cvec((L - m) % L)));
      }
  }
  sv->pc.twist = circ ? 1 : 0;
  CT_TRY_HIP(hipMemcpyAsync(sv->pc.d_mult, tab.data(), sizeof(float) * tab.size(),
                            hipMemcpyHostToDevice, st));
  std::fill(img.begin(), img.end(), 0.f);
  img[0] = 1.f;
  CT_TRY_HIP(hipMemcpyAsync(sv->u, img.data(), sizeof(float) * nn, hipMemcpyHostToDevice, st));
  CT_TRY(launch_apply_mult(&sv->pc, sv->pc.d_mult, sv->u, nullptr, sv->utmp, st));
  std::vector<float> kh(nn);
  CT_TRY_HIP(hipMemcpyAsync(kh.data(), sv->utmp, sizeof(float) * nn, hipMemcpyDeviceToHost, st));
  CT_TRY_HIP(hipStreamSynchronize(st));
  // F(K) on the multiplier grid.  Impulse response: the output image holds
  // F(k) at (x-freq i, y-freq j).  Circulant: it holds F_L(k) at vector index
  // j + n i, and grid point (k1, k2) is frequency q = k1 + n k2.
  std::vector<double> fK((size_t)half * n);
  const double L = (double)n * n;
  for (int k1 = 0; k1 < half; ++k1) {
    const double s1 = std::sin(M_PI * k1 / n);
    for (int k2 = 0; k2 < n; ++k2) {
      double fk, lap;
      if (!circ) {
        const double s2 = std::sin(M_PI * k2 / n);
        fk = (double)kh[(size_t)k2 * n + k1];
        lap = 4.0 * s1 * s1 + 4.0 * s2 * s2;
      } else {
        const double q = (double)k1 + (double)n * k2;
        fk = (double)kh[(size_t)k1 * n + k2];
        lap = 4.0 - 2.0 * std::cos(2.0 * M_PI * q / L) - 2.0 * std::cos(2.0 * M_PI * q / n);
      }
      const double v = sig * sig * fk + st2 * lap;
      if (!(v > 0.0) || !std::isfinite(v)) {
        set_error("ct_solver_create: kernel preconditioner symbol F(K) is not positive");
        return CT_E_UNSUPPORTED;
      }
      fK[(size_t)k1 * n + k2] = v;
    }
  }
  const double inv_nn = 1.0 / ((double)n * (double)n);
  if (prm->c > 0) {
    sv->c = prm->c;
  } else {
    // lambda_max(M_K^{-1/2} T M_K^{-1/2}), T = sigma^2 A^* A - (sigma tau)^2 div nabla
    for (size_t q = 0; q < tab.size(); ++q) tab[q] = (float)(inv_nn / std::sqrt(fK[q]));
    CT_TRY_HIP(hipMemcpyAsync(sv->pc.d_mult, tab.data(), sizeof(float) * tab.size(),
                              hipMemcpyHostToDevice, st));
    if (prm->start_precond)
      CT_TRY_HIP(hipMemcpyAsync(sv->u, prm->start_precond, sizeof(float) * nn,
                                hipMemcpyDeviceToDevice, st));
    else {
      auto h0 = default_start(n);
      CT_TRY_HIP(hipMemcpyAsync(sv->u, h0.data(), sizeof(float) * nn, hipMemcpyHostToDevice, st));
    }
    CT_TRY_HIP(hipStreamSynchronize(st));
    const float inv_h = (float)(1.0 / p->g.h);
    auto op = [&](float *xin, float *yout) -> int {
      CT_TRY(launch_apply_mult(&sv->pc, sv->pc.d_mult, xin, nullptr, sv->u_next, st));
      CT_TRY(launch_radon_fwd(p, sv->u_next, sv->rraw, st));
      CT_TRY(launch_grad(n, inv_h, sv->u_next, sv->w, st));
      CT_TRY(launch_radon_adj(p, sv->rraw, sv->w, (float)(sig * sig / (sv->beta * sv->beta)),
                              (float)(-st2), sv->u_next, st, 1, sv->bp_part, sv->bp_S));
      return launch_apply_mult(&sv->pc, sv->pc.d_mult, sv->u_next, nullptr, yout, st);
    };
    double lam = 0;
    CT_TRY(power_iterate(n, prm->power_iters, sv->u, sv->utmp, sv->d_red, sv->red_cap,
                         sv->d_out, op, st, &lam));
    sv->c = prm->c_safety * lam;
  }
  if (!(sv->c > 0) || !std::isfinite(sv->c)) {
    set_error("ct_solver_create: preconditioner constant is zero or non-finite");
    return CT_E_INVALID;
  }
  for (size_t q = 0; q < tab.size(); ++q) tab[q] = (float)(inv_nn / (sv->c * fK[q]));
  CT_TRY_HIP(hipMemcpyAsync(sv->pc.d_mult, tab.data(), sizeof(float) * tab.size(),
                            hipMemcpyHostToDevice, st));
  CT_TRY_HIP(hipStreamSynchronize(st));
  return CT_OK;
}

static int solver_setup(ct_solver *sv, const ct_problem *probs, const ct_params *prm,
                        hipStream_t st) {
  ct_plan *p = sv->plan;
  const int n = sv->n, N = sv->N, M = sv->M, nb = sv->nb;
  const size_t nn = (size_t)n * n, NM = (size_t)N * M;
  const size_t MW = (size_t)(M + 31) / 32;
  CT_TRY(solver_alloc(sv));
  // the set-up's backprojections use the plan's default kernel and slice
  // count; the tuning at the end decides for the iterations
  if (prm->flags & CT_FLAG_NONNEG) CT_TRY_HIP(hipMalloc(&sv->ubar, sizeof(float) * nn * nb));
  if (sv->method == CT_METHOD_CP) CT_TRY_HIP(hipMalloc(&sv->ucp, sizeof(float) * nn * nb));
  if (sv->method == CT_METHOD_ADMM) {
    for (float **b : {&sv->cg_r, &sv->cg_z, &sv->cg_p, &sv->cg_Hp})
      CT_TRY_HIP(hipMalloc(b, sizeof(float) * nn));
    CT_TRY_HIP(hipMalloc(&sv->d_cg, sizeof(double) * (4 + dot_partials_needed())));
  }
  CT_TRY(solver_set_slices(sv, p->bp_slices));
  for (int b = 0; b < nb; ++b) {
    uint32_t *mb = sv->mask + (size_t)b * N * MW;
    if (probs[b].mask)
      CT_TRY_HIP(hipMemcpyAsync(mb, probs[b].mask, sizeof(uint32_t) * N * MW,
                                hipMemcpyDeviceToDevice, st));
    else
      CT_TRY_HIP(hipMemsetAsync(mb, 0, sizeof(uint32_t) * N * MW, st));
  }
  if (prm->flags & CT_FLAG_VALIDATE) {
    int *flag = reinterpret_cast<int *>(sv->d_out);
    CT_TRY_HIP(hipMemsetAsync(flag, 0, sizeof(int), st));
    bool finite = true;
    for (int b = 0; b < nb; ++b) {
      CT_TRY(launch_nonfinite(probs[b].sino, (int64_t)NM, flag, st));
      if (probs[b].bound) CT_TRY(launch_nonfinite(probs[b].bound, (int64_t)NM, flag, st));
      finite = finite && std::isfinite(probs[b].bound_scalar);
    }
    int hflag = 0;
    CT_TRY_HIP(hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, st));
    CT_TRY_HIP(hipStreamSynchronize(st));
    if (hflag || !finite) {
      set_error("ct_solver_create: non-finite value in sinogram or bound");
      return CT_E_NONFINITE;
    }
  }
  CT_TRY(precond_init(&sv->pc, n, prm->sigma, prm->tau, -1.0, prm->eps));
  double *d_norm = sv->d_out;
  // beta = ||R_h|| (§5.1 normalization; power iteration unless given).  It and
  // c depend on the geometry only, so one estimate serves the whole batch.
  if (prm->beta > 0) {
    sv->beta = prm->beta;
  } else {
    if (prm->start_norm)
      CT_TRY_HIP(hipMemcpyAsync(sv->u, prm->start_norm, sizeof(float) * nn,
                                hipMemcpyDeviceToDevice, st));
    else {
      auto h0 = default_start(n);
      CT_TRY_HIP(hipMemcpyAsync(sv->u, h0.data(), sizeof(float) * nn, hipMemcpyHostToDevice, st));
      CT_TRY_HIP(hipStreamSynchronize(st));
    }
    auto op = [&](float *xin, float *yout) -> int {
      CT_TRY(launch_radon_fwd(p, xin, sv->rraw, st));
      return launch_radon_adj(p, sv->rraw, nullptr, 1.0f, 0.0f, yout, st, 1, sv->bp_part,
                              sv->bp_S);
    };
    double lam = 0;
    CT_TRY(power_iterate(n, prm->power_iters, sv->u, sv->utmp, sv->d_red, sv->red_cap, d_norm,
                         op, st, &lam));
    sv->beta = std::sqrt(lam);
  }
  if (!(sv->beta > 0) || !std::isfinite(sv->beta)) {
    set_error("ct_solver_create: operator norm estimate is zero or non-finite");
    return CT_E_INVALID;
  }
  const int pkind = (int)((prm->flags >> CT_PRECOND_SHIFT) & 15u);
  if (pkind == CT_PRECOND_IMPULSE || pkind == CT_PRECOND_CIRCULANT) {
    CT_TRY(kernel_precond_setup(sv, prm, pkind == CT_PRECOND_CIRCULANT, st));
  } else {
  // c > lambda_max(tilde M^{-1} A^* A) (§4.3.1), by power iteration on
  // tilde M^{-1/2} A^* A tilde M^{-1/2} unless given
  if (prm->c > 0) {
    sv->c = prm->c;
  } else {
    auto tab = multiplier_table(n, prm->sigma, prm->tau, 1.0, prm->eps, true);
    CT_TRY_HIP(hipMemcpyAsync(sv->pc.d_mult, tab.data(), sizeof(float) * tab.size(),
                              hipMemcpyHostToDevice, st));
    CT_TRY_HIP(hipStreamSynchronize(st));
    if (prm->start_precond)
      CT_TRY_HIP(hipMemcpyAsync(sv->u, prm->start_precond, sizeof(float) * nn,
                                hipMemcpyDeviceToDevice, st));
    else {
      auto h0 = default_start(n);
      CT_TRY_HIP(hipMemcpyAsync(sv->u, h0.data(), sizeof(float) * nn, hipMemcpyHostToDevice, st));
      CT_TRY_HIP(hipStreamSynchronize(st));
    }
    const float inv_b2 = (float)(1.0 / (sv->beta * sv->beta));
    auto op = [&](float *xin, float *yout) -> int {
      CT_TRY(launch_apply_mult(&sv->pc, sv->pc.d_mult, xin, nullptr, sv->u_next, st));
      CT_TRY(launch_radon_fwd(p, sv->u_next, sv->rraw, st));
      CT_TRY(launch_radon_adj(p, sv->rraw, nullptr, inv_b2, 0.0f, sv->u_next, st, 1,
                              sv->bp_part, sv->bp_S));
      return launch_apply_mult(&sv->pc, sv->pc.d_mult, sv->u_next, nullptr, yout, st);
    };
    double lam = 0;
    CT_TRY(power_iterate(n, prm->power_iters, sv->u, sv->utmp, sv->d_red, sv->red_cap, d_norm,
                         op, st, &lam));
    sv->c = prm->c_safety * lam;
  }
  if (!(sv->c > 0) || !std::isfinite(sv->c)) {
    set_error("ct_solver_create: preconditioner constant is zero or non-finite");
    return CT_E_INVALID;
  }
  sv->pc.c = sv->c;
  sv->rich_m = 1.1 * (sv->sigma * sv->sigma +
                      8.0 * (sv->sigma * sv->tau) * (sv->sigma * sv->tau) / (p->g.h * p->g.h));
  {
    // PDRQS2 (§4.3.1 with Q = A^* A): rho / (sigma c + (sigma tau)^2 lambda_Delta rho)
    // ADMM (§4.6): rho / (c + tau^2 lambda_Delta rho), i.e. the table at sigma = 1
    const double csig = sv->method == CT_METHOD_PDRQS2 ? sv->c / sv->sigma : sv->c;
    const double sig_m = sv->method == CT_METHOD_ADMM ? 1.0 : sv->sigma;
    auto m = multiplier_table(n, sig_m, sv->tau, csig, sv->eps, false, sv->ubar != nullptr);
    CT_TRY_HIP(hipMemcpyAsync(sv->pc.d_mult, m.data(), sizeof(float) * m.size(),
                              hipMemcpyHostToDevice, st));
    CT_TRY_HIP(hipStreamSynchronize(st));
  }
  }
  sv->pc.c = sv->c;
  for (int b = 0; b < nb; ++b)
    CT_TRY(launch_build_target(N, M, probs[b].sino, probs[b].bound, probs[b].bound_scalar,
                               sv->mask + (size_t)b * N * MW, (float)(1.0 / sv->beta),
                               sv->target + (size_t)b * NM, st));
  sv->lam_t = probs[0].lambda / (sv->beta * sv->beta);
  CT_TRY(solver_zero_state(sv, st));
  CT_TRY(solver_tune(sv, prm, st));
  CT_TRY_HIP(hipStreamSynchronize(st));
  return CT_OK;
}

// Capture 2 npairs iterations of every solver in svs (all at the same
// ping-pong parity) as one HIP graph on a private stream, the last in mode
// last_mode (0, or 2 to keep y1, w and A u for a record); the pointers are
// back in place after them.
static int capture_pairs(ct_solver *const *svs, int count, hipStream_t cap, int npairs,
                         int last_mode, hipGraphExec_t *out) {
  hipGraph_t graph = nullptr;
  CT_TRY_HIP(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
  int rc = CT_OK;
  const int n_it = 2 * npairs;
  for (int it = 0; it < n_it && rc == CT_OK; ++it)
    for (int q = 0; q < count && rc == CT_OK; ++q) {
      const int64_t it0 = svs[q]->iters;
      rc = solver_iter(svs[q], it == n_it - 1 ? last_mode : 0, cap);
      svs[q]->iters = it0;  // nothing ran
    }
  hipError_t e = hipStreamEndCapture(cap, &graph);
  if (rc != CT_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return rc;
  }
  CT_TRY_HIP(e);
  hipError_t ei = hipGraphInstantiate(out, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  CT_TRY_HIP(ei);
  // its first launch then finds it on the device already
  CT_TRY_HIP(hipGraphUpload(*out, cap));
  CT_TRY_HIP(hipStreamSynchronize(cap));
  return CT_OK;
}


// Captures every graph multi_step replays: the three kinds at both ping-pong
// parities (the other parity with u and u_next exchanged for its capture and
// restored after), so that no later step spends its time capturing.
static int prepare_graphs(ct_solver *const *svs, int count, hipStream_t *cap,
                          hipGraphExec_t graphs[kGraphSlots], float *graph_u[kGraphSlots]) {
  bool all = true;
  for (int i = 0; i < kGraphSlots; ++i) all = all && graphs[i] != nullptr;
  if (all) return CT_OK;
  if (!*cap) CT_TRY_HIP(hipStreamCreateWithFlags(cap, hipStreamNonBlocking));
  for (int side = 0; side < 2; ++side) {
    if (side == 1)
      for (int q = 0; q < count; ++q) std::swap(svs[q]->u, svs[q]->u_next);
    const int parity = (svs[0]->u < svs[0]->u_next) ? 0 : 1;
    int rc = CT_OK;
    for (int kind = 0; kind < 3 && rc == CT_OK; ++kind) {
      const int idx = parity + 2 * kind;
      if (graphs[idx]) continue;
      rc = capture_pairs(svs, count, *cap, kind == 2 ? kLongPairs : 1, kind == 1 ? 2 : 0,
                         &graphs[idx]);
      if (rc == CT_OK) graph_u[idx] = svs[0]->u;
    }
    if (side == 1)
      for (int q = 0; q < count; ++q) std::swap(svs[q]->u, svs[q]->u_next);
    CT_TRY(rc);
  }
  return CT_OK;
}

// k iterations of every solver in svs (same iteration count and parity).
// With k >= 3 they replay from HIP graphs: an odd k first runs one iteration
// eagerly; the last pair is the graph whose second iteration keeps y1, w and
// A u for a record; the pairs before it run kLongPairs at a time from the
// long graph, the rest from the plain two-iteration graph (the same
// launches in the same order as eager steps).  Smaller k run eagerly, the
// last in mode 2.  graphs[kGraphSlots] and cap are the caller's cache, all
// captured by the first call with k > 0 (prepare_graphs).
static int multi_step(ct_solver *const *svs, int count, int k, hipStream_t st, hipStream_t *cap,
                      hipGraphExec_t graphs[kGraphSlots], float *graph_u[kGraphSlots]) {
  int left = k;
  bool graphs_ok = true;
  for (int q = 0; q < count; ++q) graphs_ok = graphs_ok && svs[q]->use_graph;
  // the first step of any length captures them all
  if (graphs_ok && k > 0) CT_TRY(prepare_graphs(svs, count, cap, graphs, graph_u));
  if (graphs_ok && left >= 3) {
    if (left & 1) {
      for (int q = 0; q < count; ++q) CT_TRY(solver_iter(svs[q], 0, st));
      left -= 1;
    }
    const int parity = (svs[0]->u < svs[0]->u_next) ? 0 : 1;
    // kind 0: a plain pair, 1: the record pair, 2: kLongPairs plain pairs
    auto graph = [&](int kind, hipGraphExec_t *g) -> int {
      const int idx = parity + 2 * kind;
      if (!graphs[idx]) {
        if (!*cap) CT_TRY_HIP(hipStreamCreateWithFlags(cap, hipStreamNonBlocking));
        CT_TRY(capture_pairs(svs, count, *cap, kind == 2 ? kLongPairs : 1, kind == 1 ? 2 : 0,
                             &graphs[idx]));
        graph_u[idx] = svs[0]->u;
      }
      if (graph_u[idx] != svs[0]->u) {
        set_error("ct_pd_step: graph parity mismatch");
        return CT_E_STATE;
      }
      *g = graphs[idx];
      return CT_OK;
    };
    const int pairs = left / 2;
    const int longs = (pairs - 1) / kLongPairs;
    const int singles = pairs - 1 - longs * kLongPairs;
    hipGraphExec_t g0 = nullptr, g2 = nullptr, gl = nullptr;
    if (longs > 0) CT_TRY(graph(2, &gl));
    if (singles > 0) CT_TRY(graph(0, &g0));
    CT_TRY(graph(1, &g2));
    for (int q = 0; q < longs; ++q) CT_TRY_HIP(hipGraphLaunch(gl, st));
    for (int q = 0; q < singles; ++q) CT_TRY_HIP(hipGraphLaunch(g0, st));
    CT_TRY_HIP(hipGraphLaunch(g2, st));
    for (int q = 0; q < count; ++q) svs[q]->iters += left;
    left = 0;
  }
  for (int it = 0; it < left; ++it)
    for (int q = 0; q < count; ++q) CT_TRY(solver_iter(svs[q], it == left - 1 ? 2 : 0, st));
  if (k > 0)
    for (int q = 0; q < count; ++q) svs[q]->have_dual = true;
  return CT_OK;
}

static int solver_create(const ct_plan *p, const ct_problem *probs, int nb, const ct_params *prm,
                         ct_stream s, ct_solver **out) {
  if (!p || !probs || !prm || !out || nb < 1) {
    set_error("ct_solver_create: null argument or empty batch");
    return CT_E_INVALID;
  }
  *out = nullptr;
  if (!(prm->sigma > 0) || !(prm->tau > 0) || !(prm->eps > 0) || prm->k_max < 0 ||
      prm->gap_every < 0 || (prm->c <= 0 && !(prm->c_safety > 0)) ||
      ((prm->c <= 0 || prm->beta <= 0) && prm->power_iters < 1)) {
    set_error("ct_solver_create: need sigma, tau, eps > 0, lambda >= 0, k_max >= 0, "
              "power_iters >= 1 when beta or c is estimated");
    return CT_E_INVALID;
  }
  for (int b = 0; b < nb; ++b) {
    const ct_problem &pr = probs[b];
    if (!pr.sino) {
      set_error("ct_solver_create: null sinogram");
      return CT_E_INVALID;
    }
    if (!(pr.lambda >= 0) || !std::isfinite(pr.lambda)) {
      set_error("ct_solver_create: need sigma, tau, eps > 0, lambda >= 0, k_max >= 0, "
                "power_iters >= 1 when beta or c is estimated");
      return CT_E_INVALID;
    }
    if (pr.lambda != probs[0].lambda) {
      set_error("ct_solver_create: the problems of one batch need the same lambda");
      return CT_E_INVALID;
    }
    if (pr.mask && !pr.bound && !std::isfinite(pr.bound_scalar)) {
      set_error("ct_solver_create: non-finite bound");
      return CT_E_INVALID;
    }
  }
  if (!fft_size_ok(p->g.n)) {
    set_error("ct_solver_create: n must be even, 2^a 3^b and <= 4096");
    return CT_E_UNSUPPORTED;
  }
  if (prm->bp_slices < 0 || prm->bp_slices > kMaxSlices || prm->tv_blocks < 0 ||
      prm->tv_blocks > 4096 ||
      (prm->bp_kernel != CT_BP_AUTO && prm->bp_kernel != CT_BP_ONE_ANGLE &&
       prm->bp_kernel != CT_BP_PAIRS4 && prm->bp_kernel != CT_BP_PAIRS8) ||
      (prm->options & ~15u) != 0 || prm->fwd_walk < 0 || prm->fwd_walk > 4 ||
      prm->fwd_walk == 3) {
    set_error("ct_solver_create: need 0 <= bp_slices <= 16, 0 <= tv_blocks <= 4096, a CT_BP_* "
              "kernel, known CT_OPT_* bits and fwd_walk 0, 1, 2 or 4");
    return CT_E_INVALID;
  }
  if ((prm->bp_kernel == CT_BP_PAIRS4 || prm->bp_kernel == CT_BP_PAIRS8) && p->n_bpp == 0) {
    set_error("ct_solver_create: mirror-pair backprojection needs angles that pair as "
              "theta, pi - theta");
    return CT_E_UNSUPPORTED;
  }
  const int method = (int)((prm->flags >> CT_METHOD_SHIFT) & 15u);
  if (method > CT_METHOD_PDRQS3) {
    set_error("ct_solver_create: unknown method");
    return CT_E_INVALID;
  }
  const int pkind = (int)((prm->flags >> CT_PRECOND_SHIFT) & 15u);
  if (pkind > CT_PRECOND_CIRCULANT) {
    set_error("ct_solver_create: unknown preconditioner");
    return CT_E_INVALID;
  }
  if (pkind != CT_PRECOND_INVNORM &&
      (method != CT_METHOD_PDRQS1 || (prm->flags & CT_FLAG_NONNEG) || (p->g.n & 1) || nb != 1)) {
    set_error("ct_solver_create: the impulse-response and circulant preconditioners are for "
              "single-problem PDRQS1 (even n)");
    return CT_E_UNSUPPORTED;
  }
  if (method == CT_METHOD_ADMM) {
    if (nb != 1) {
      set_error("ct_solver_create: ADMM runs one problem per solver");
      return CT_E_UNSUPPORTED;
    }
    if (probs[0].mask) {
      set_error("ct_solver_create: ADMM solves the unconstrained problem (no D0)");
      return CT_E_UNSUPPORTED;
    }
  }
  if (method != CT_METHOD_PDRQS1 && method != CT_METHOD_RICHARDSON &&
      (prm->flags & CT_FLAG_NONNEG)) {
    set_error("ct_solver_create: u >= 0 is available for PDRQS1 only");
    return CT_E_UNSUPPORTED;
  }
  if (method == CT_METHOD_PDRQS2)
    for (int b = 0; b < nb; ++b)
      if (probs[b].mask) {
        set_error("ct_solver_create: PDRQS2 solves the unconstrained problem (no D0)");
        return CT_E_UNSUPPORTED;
      }
  ct_solver *sv = new (std::nothrow) ct_solver();
  if (!sv) return CT_E_DEVICE;
  sv->plan = const_cast<ct_plan *>(p);
  sv->fwd = p;
  sv->nb = nb;
  sv->method = method;
  sv->n = p->g.n;
  sv->N = p->g.n_angles;
  sv->M = p->g.n_bins;
  sv->sigma = prm->sigma;
  sv->tau = prm->tau;
  sv->eps = prm->eps;
  sv->options = prm->options;
  sv->use_graph = !(prm->options & CT_OPT_NO_GRAPH);
  sv->defer_combine = !(prm->options & CT_OPT_NO_DEFER);
  sv->fuse_tv = !(prm->options & CT_OPT_SEPARATE_TV);
  int rc = solver_setup(sv, probs, prm, S(s));
  if (rc != CT_OK) {
    (void)hipStreamSynchronize(S(s));
    solver_free(sv);
    delete sv;
    return rc;
  }
  *out = sv;
  return CT_OK;
}

// FP64 record of problem b (see ct_gap).
static int solver_gap(ct_solver *sv, int b, double out[6], hipStream_t st) {
  const size_t nn = (size_t)sv->n * sv->n, NM = (size_t)sv->N * sv->M;
  const size_t MW = (size_t)(sv->M + 31) / 32;
  double *o = sv->d_out;
  CT_TRY(launch_sino_gap(sv->N, sv->M, sv->r + b * NM, sv->y1 + b * NM, sv->target + b * NM,
                         sv->mask + b * (size_t)sv->N * MW, sv->d_red, sv->red_cap, o, st));
  // z = A^* y1 - tau div w  (= K^* y), into the first u_tmp image
  CT_TRY(launch_radon_adj(sv->plan, sv->y1 + b * NM, sv->w + b * 2 * nn,
                          (float)(1.0 / sv->beta), (float)(-sv->tau), sv->utmp, st, 1,
                          sv->bp_part, sv->bp_S, sv->bp_kern));
  CT_TRY(launch_img_gap(sv->n, (float)(1.0 / sv->plan->g.h), sv->u + b * nn,
                        sv->u_next + b * nn, sv->utmp, sv->d_red, sv->red_cap, o + 3, st));
  double h[6];
  CT_TRY_HIP(hipMemcpyAsync(h, o, sizeof(double) * 6, hipMemcpyDeviceToHost, st));
  CT_TRY_HIP(hipStreamSynchronize(st));
  const double P = h[0] + sv->lam_t * h[3];
  out[0] = P;
  out[1] = h[1];
  out[2] = P + h[1];
  out[3] = std::sqrt(h[5]);
  out[4] = h[2];
  out[5] = std::sqrt(h[4]);
  return CT_OK;
}

extern "C" {

int ct_solver_create(const ct_plan *p, const ct_problem *prob, const ct_params *prm,
                     ct_stream s, ct_solver **out) {
  clear_error();
  return solver_create(p, prob, 1, prm, s, out);
}

int ct_solver_create_batch(const ct_plan *p, const ct_problem *probs, int32_t nb,
                           const ct_params *prm, ct_stream s, ct_solver **out) {
  clear_error();
  return solver_create(p, probs, nb, prm, s, out);
}

int ct_solver_destroy(ct_solver *sv) {
  clear_error();
  if (!sv) return CT_OK;
  solver_free(sv);
  delete sv;
  return CT_OK;
}

int ct_solver_info(const ct_solver *sv, double out[4]) {
  clear_error();
  if (!sv || !out) {
    set_error("ct_solver_info: null argument");
    return CT_E_INVALID;
  }
  out[0] = sv->beta;
  out[1] = sv->c;
  out[2] = sv->lam_t;
  out[3] = (double)sv->iters;
  return CT_OK;
}

int ct_solver_layout(const ct_solver *sv, int32_t out[6]) {
  clear_error();
  if (!sv || !out) {
    set_error("ct_solver_layout: null argument");
    return CT_E_INVALID;
  }
  out[0] = sv->nb;
  out[1] = sv->bp_S;
  out[2] = sv->fwd->slots;
  out[3] = sv->fwd->n_groups;
  const bool pairs = sv->plan->n_bpp > 0 && sv->bp_kern != 0;
  out[4] = pairs ? 2 : 1;
  out[5] = pairs ? sv->bp_kern : 0;
  return CT_OK;
}

int ct_solver_tuning(const ct_solver *sv, int32_t out[4]) {
  clear_error();
  if (!sv || !out) {
    set_error("ct_solver_tuning: null argument");
    return CT_E_INVALID;
  }
  out[0] = sv->tune_source;
  out[1] = sv->tune_timed;
  out[2] = sv->fuse_tv ? sv->tv_blocks : 0;
  out[3] = sv->tune_saved;
  return CT_OK;
}

int ct_solver_set_fit(ct_solver *sv, int32_t fit, const float *aux, ct_stream s) {
  clear_error();
  if (!sv || fit < CT_FIT_STANDARD || fit > CT_FIT_HARD) {
    set_error("ct_solver_set_fit: invalid argument");
    return CT_E_INVALID;
  }
  if (sv->method != CT_METHOD_PDRQS1 && sv->method != CT_METHOD_RICHARDSON) {
    set_error("ct_solver_set_fit: the data-term variants are for PDRQS1");
    return CT_E_UNSUPPORTED;
  }
  if (sv->iters != 0 || has_graphs(sv)) {
    set_error("ct_solver_set_fit: set the data term before the first iteration");
    return CT_E_STATE;
  }
  const bool needs_aux = fit == CT_FIT_WEIGHTED || fit == CT_FIT_EVERYWHERE;
  if (needs_aux && !aux) {
    set_error("ct_solver_set_fit: this data term needs its per-bin array");
    return CT_E_INVALID;
  }
  hipStream_t st = S(s);
  const size_t NM = (size_t)sv->N * sv->M * sv->nb;
  if (needs_aux) {
    if (!sv->fit_aux) CT_TRY_HIP(hipMalloc(&sv->fit_aux, sizeof(float) * NM));
    if (fit == CT_FIT_EVERYWHERE) {
      // b = u0 / beta on every bin
      const double beta = sv->beta;
      CT_TRY_HIP(hipMemcpyAsync(sv->d_out, &beta, sizeof(double), hipMemcpyHostToDevice, st));
      CT_TRY(launch_scale_by_inv(aux, (int64_t)NM, sv->d_out, sv->fit_aux, st));
    } else {
      CT_TRY_HIP(hipMemcpyAsync(sv->fit_aux, aux, sizeof(float) * NM, hipMemcpyDeviceToDevice,
                                st));
    }
    CT_TRY_HIP(hipStreamSynchronize(st));
  }
  sv->fit = fit;
  return CT_OK;
}

int ct_solver_set_admm(ct_solver *sv, int32_t cg_steps, double mu) {
  clear_error();
  if (!sv || cg_steps < 1 || cg_steps > 64 || !(mu > 0) || !std::isfinite(mu)) {
    set_error("ct_solver_set_admm: need 1 <= cg_steps <= 64 and mu > 0");
    return CT_E_INVALID;
  }
  if (sv->method != CT_METHOD_ADMM) {
    set_error("ct_solver_set_admm: not an ADMM solver");
    return CT_E_UNSUPPORTED;
  }
  if (sv->iters != 0 || has_graphs(sv)) {
    set_error("ct_solver_set_admm: set the options before the first iteration");
    return CT_E_STATE;
  }
  sv->admm_cg = cg_steps;
  sv->admm_mu = mu;
  return CT_OK;
}

int ct_pd_step(ct_solver *sv, int32_t k, ct_stream s) {
  clear_error();
  if (!sv || k < 0) {
    set_error("ct_pd_step: invalid argument");
    return CT_E_INVALID;
  }
  if (!sv->use_graph) {
    for (int it = 0; it < k; ++it) CT_TRY(solver_iter(sv, it == k - 1 ? 2 : 0, S(s)));
    if (k > 0) sv->have_dual = true;
    return CT_OK;
  }
  ct_solver *one[1] = {sv};
  return multi_step(one, 1, k, S(s), &sv->cap_stream, sv->gexec, sv->gexec_u);
}

int ct_pd_step_timed(ct_solver *sv, int32_t k, double ms_out[5], ct_stream s) {
  clear_error();
  if (!sv || k < 1 || !ms_out) {
    set_error("ct_pd_step_timed: invalid argument");
    return CT_E_INVALID;
  }
  if (sv->method == CT_METHOD_ADMM) {
    set_error("ct_pd_step_timed: the phase split is that of the PDRQ iterations");
    return CT_E_UNSUPPORTED;
  }
  hipStream_t st = S(s);
  hipEvent_t ev[5] = {};
  int rc = CT_OK;
  for (int i = 0; i < 5 && rc == CT_OK; ++i)
    if (hipEventCreate(&ev[i]) != hipSuccess) rc = CT_E_DEVICE;
  for (int i = 0; i < 5; ++i) ms_out[i] = 0.0;
  for (int it = 0; it < k && rc == CT_OK; ++it) {
    rc = solver_iter(sv, it == k - 1 ? 2 : 0, st, ev);
    if (rc == CT_OK && hipEventSynchronize(ev[4]) != hipSuccess) rc = CT_E_DEVICE;
    for (int i = 0; i < 4 && rc == CT_OK; ++i) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, ev[i], ev[i + 1]) != hipSuccess) rc = CT_E_DEVICE;
      ms_out[i] += ms;
      ms_out[4] += ms;
    }
  }
  for (int i = 0; i < 5; ++i)
    if (ev[i]) (void)hipEventDestroy(ev[i]);
  if (rc == CT_E_DEVICE) set_error("ct_pd_step_timed: HIP event failure");
  if (rc == CT_OK) {
    sv->have_dual = true;
    for (int i = 0; i < 5; ++i) ms_out[i] /= k;
  }
  return rc;
}

int ct_state_export(const ct_solver *sv, float *u, float *vb1, float *vb2, ct_stream s) {
  clear_error();
  if (!sv) {
    set_error("ct_state_export: null solver");
    return CT_E_INVALID;
  }
  const size_t nn = (size_t)sv->n * sv->n * sv->nb, NM = (size_t)sv->N * sv->M * sv->nb;
  hipStream_t st = S(s);
  if (u) CT_TRY_HIP(hipMemcpyAsync(u, sv->u, sizeof(float) * nn, hipMemcpyDeviceToDevice, st));
  if (vb1)
    CT_TRY_HIP(hipMemcpyAsync(vb1, sv->vb1, sizeof(float) * NM, hipMemcpyDeviceToDevice, st));
  if (vb2)
    CT_TRY_HIP(hipMemcpyAsync(vb2, sv->vb2, sizeof(float) * nn * 2, hipMemcpyDeviceToDevice, st));
  return CT_OK;
}

int ct_state_export_ubar(const ct_solver *sv, float *ubar, ct_stream s) {
  clear_error();
  if (!sv || !ubar) {
    set_error("ct_state_export_ubar: null argument");
    return CT_E_INVALID;
  }
  if (!sv->ubar) {
    set_error("ct_state_export_ubar: the solver has no u >= 0 constraint");
    return CT_E_STATE;
  }
  const size_t nn = (size_t)sv->n * sv->n * sv->nb;
  CT_TRY_HIP(hipMemcpyAsync(ubar, sv->ubar, sizeof(float) * nn, hipMemcpyDeviceToDevice, S(s)));
  return CT_OK;
}

int ct_state_import_ubar(ct_solver *sv, const float *ubar, ct_stream s) {
  clear_error();
  if (!sv || !ubar) {
    set_error("ct_state_import_ubar: null argument");
    return CT_E_INVALID;
  }
  if (!sv->ubar) {
    set_error("ct_state_import_ubar: the solver has no u >= 0 constraint");
    return CT_E_STATE;
  }
  const size_t nn = (size_t)sv->n * sv->n * sv->nb;
  CT_TRY_HIP(hipMemcpyAsync(sv->ubar, ubar, sizeof(float) * nn, hipMemcpyDeviceToDevice, S(s)));
  return CT_OK;
}

int ct_state_import(ct_solver *sv, const float *u, const float *vb1, const float *vb2,
                    ct_stream s) {
  clear_error();
  if (!sv || !u || !vb1 || !vb2) {
    set_error("ct_state_import: null argument");
    return CT_E_INVALID;
  }
  if (sv->method == CT_METHOD_ADMM) {
    set_error("ct_state_import: an ADMM state also holds z (not importable)");
    return CT_E_UNSUPPORTED;
  }
  const size_t nn = (size_t)sv->n * sv->n * sv->nb, NM = (size_t)sv->N * sv->M * sv->nb;
  hipStream_t st = S(s);
  CT_TRY_HIP(hipMemcpyAsync(sv->u, u, sizeof(float) * nn, hipMemcpyDeviceToDevice, st));
  CT_TRY_HIP(hipMemcpyAsync(sv->vb1, vb1, sizeof(float) * NM, hipMemcpyDeviceToDevice, st));
  CT_TRY_HIP(hipMemcpyAsync(sv->vb2, vb2, sizeof(float) * nn * 2, hipMemcpyDeviceToDevice, st));
  if (sv->method == CT_METHOD_CP) {
    // restart of Algorithm CP: the extrapolated iterate is u itself
    CT_TRY_HIP(hipMemcpyAsync(sv->ucp, u, sizeof(float) * nn, hipMemcpyDeviceToDevice, st));
    sv->have_dual = false;
    return CT_OK;
  }
  // caches: s1 = vb1 + sigma A u (PDRQS2: b - A u), s2 = vb2 + sigma tau nabla u
  const SinoEpi ep{(float)(1.0 / sv->beta), (float)sv->sigma, sv->target, sv->mask, sv->vb1,
                   sv->s1, nullptr, nullptr,
                   sv->method == CT_METHOD_PDRQS2 ? 5 : (sv->method == CT_METHOD_PDRQS3 ? 8 : 1)};
  CT_TRY(launch_radon_fwd(sv->fwd, sv->u, nullptr, st, &ep, sv->nb));
  CT_TRY(launch_tv_update(sv->n, (float)(1.0 / sv->plan->g.h), sv->u,
                          (float)(sv->sigma * sv->tau), 0.0f, sv->vb2, sv->s2, nullptr, 1, st,
                          sv->nb));
  sv->have_dual = false;
  return CT_OK;
}

int ct_gap(ct_solver *sv, double *out, ct_stream s) {
  clear_error();
  if (!sv || !out) {
    set_error("ct_gap: null argument");
    return CT_E_INVALID;
  }
  if (!sv->have_dual) {
    set_error("ct_gap: no iteration since creation or import");
    return CT_E_STATE;
  }
  if (sv->method == CT_METHOD_CP || sv->method == CT_METHOD_PDRQS2 ||
      sv->method == CT_METHOD_ADMM || sv->method == CT_METHOD_PDRQS3 ||
      sv->fit != CT_FIT_STANDARD) {
    set_error("ct_gap: the record is defined for PDRQS1 with the standard data term");
    return CT_E_UNSUPPORTED;
  }
  for (int b = 0; b < sv->nb; ++b) CT_TRY(solver_gap(sv, b, out + 6 * b, S(s)));
  return CT_OK;
}

}  // extern "C"

struct ct_group {
  std::vector<ct_solver *> svs;
  hipStream_t cap = nullptr;
  hipGraphExec_t graphs[kGraphSlots] = {};
  float *graph_u[kGraphSlots] = {};
  ~ct_group() {
    for (auto g : graphs)
      if (g) (void)hipGraphExecDestroy(g);
    if (cap) (void)hipStreamDestroy(cap);
  }
};

extern "C" {

int ct_group_create(ct_solver *const *svs, int32_t count, ct_group **out) {
  clear_error();
  if (!svs || count < 1 || !out) {
    set_error("ct_group_create: null argument or empty group");
    return CT_E_INVALID;
  }
  *out = nullptr;
  for (int q = 0; q < count; ++q) {
    if (!svs[q]) {
      set_error("ct_group_create: null solver");
      return CT_E_INVALID;
    }
    if (svs[q]->iters != svs[0]->iters) {
      set_error("ct_group_create: solvers must have done the same number of iterations");
      return CT_E_STATE;
    }
    for (int r = 0; r < q; ++r)
      if (svs[r] == svs[q]) {
        set_error("ct_group_create: a solver appears twice");
        return CT_E_INVALID;
      }
  }
  ct_group *g = new (std::nothrow) ct_group();
  if (!g) return CT_E_DEVICE;
  g->svs.assign(svs, svs + count);
  *out = g;
  return CT_OK;
}

int ct_group_step(ct_group *g, int32_t k, ct_stream s) {
  clear_error();
  if (!g || k < 0) {
    set_error("ct_group_step: invalid argument");
    return CT_E_INVALID;
  }
  for (ct_solver *sv : g->svs)
    if (sv->iters != g->svs[0]->iters) {
      set_error("ct_group_step: a solver of the group was stepped on its own");
      return CT_E_STATE;
    }
  return multi_step(g->svs.data(), (int)g->svs.size(), k, S(s), &g->cap, g->graphs,
                    g->graph_u);
}

int ct_group_destroy(ct_group *g) {
  clear_error();
  delete g;
  return CT_OK;
}

int ct_reconstruct(const ct_plan *p, const ct_problem *prob, const ct_params *prm, float *u_out,
                   double *report, int32_t report_len, ct_stream s) {
  clear_error();
  if (!u_out || !prm) {
    set_error("ct_reconstruct: null argument");
    return CT_E_INVALID;
  }
  float *outs[1] = {u_out};
  return ct_reconstruct_batched(1, &p, prob, prm, outs, report, report_len, s);
}

int ct_reconstruct_batched(int32_t count, const ct_plan *const *plans, const ct_problem *probs,
                           const ct_params *prm, float *const *u_out, double *report,
                           int32_t report_len, ct_stream s) {
  clear_error();
  if (count < 1 || !plans || !probs || !prm || !u_out) {
    set_error("ct_reconstruct_batched: null argument or empty batch");
    return CT_E_INVALID;
  }
  for (int i = 0; i < count; ++i)
    if (!plans[i] || !u_out[i]) {
      set_error("ct_reconstruct_batched: null plan or output");
      return CT_E_INVALID;
    }
  hipStream_t st = S(s);
  // one solver per (plan, lambda): its problems share every kernel launch
  std::vector<std::vector<int>> groups;
  for (int i = 0; i < count; ++i) {
    bool placed = false;
    for (auto &g : groups)
      if (plans[g[0]] == plans[i] && probs[g[0]].lambda == probs[i].lambda) {
        g.push_back(i);
        placed = true;
        break;
      }
    if (!placed) groups.push_back({i});
  }
  struct Owned : ct_group {
    ~Owned() {
      for (auto sv : svs) ct_solver_destroy(sv);
    }
  } own;
  for (auto &g : groups) {
    std::vector<ct_problem> pg;
    for (int i : g) pg.push_back(probs[i]);
    ct_solver *sv = nullptr;
    CT_TRY(solver_create(plans[g[0]], pg.data(), (int)pg.size(), prm, s, &sv));
    own.svs.push_back(sv);
  }
  const int ng = (int)own.svs.size();
  const int n_rec = prm->gap_every > 0 ? prm->k_max / prm->gap_every : 0;
  int done = 0, rec = 0;
  while (done < prm->k_max) {
    const int k = (n_rec > 0 && report) ? std::min(prm->gap_every, prm->k_max - done)
                                        : prm->k_max - done;
    CT_TRY(multi_step(own.svs.data(), ng, k, st, &own.cap, own.graphs, own.graph_u));
    done += k;
    if (n_rec > 0 && report && k == prm->gap_every) {
      for (int gi = 0; gi < ng; ++gi)
        for (int b = 0; b < (int)groups[gi].size(); ++b) {
          const int i = groups[gi][b];
          const int64_t at = ((int64_t)i * n_rec + rec) * 6;
          if (at + 6 > report_len) continue;
          double r6[6];
          CT_TRY(solver_gap(own.svs[gi], b, r6, st));
          for (int q = 0; q < 6; ++q) {
            report[at + q] = r6[q];
            if (!std::isfinite(r6[q])) {
              set_error("ct_reconstruct: gap record is not finite");
              return CT_E_DIVERGED;
            }
          }
        }
      ++rec;
    }
  }
  for (int gi = 0; gi < ng; ++gi) {
    ct_solver *sv = own.svs[gi];
    const size_t nn = (size_t)sv->n * sv->n;
    for (int b = 0; b < (int)groups[gi].size(); ++b)
      CT_TRY_HIP(hipMemcpyAsync(u_out[groups[gi][b]], sv->u + b * nn, sizeof(float) * nn,
                                hipMemcpyDeviceToDevice, st));
  }
  CT_TRY_HIP(hipStreamSynchronize(st));
  return CT_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Unrolled PDRQS1 with a reverse sweep (derivatives of u_K with respect to the
// data u0 and the weight lambda), checkpointing every `every` iterations.

struct ct_tape {
  ct_solver *sv = nullptr;
  int K = 0, every = 0, n_ck = 0;
  int64_t iters_after = 0;
  std::vector<float *> bufs;  // everything below, freed together
  std::vector<float *> ck;    // per checkpoint: u, vb1, vb2 (3 entries each)
  float *q1s = nullptr, *q2s = nullptr;
  float *U = nullptr, *Utot = nullptr, *X = nullptr, *V1 = nullptr, *P = nullptr,
        *Q1 = nullptr, *bbar = nullptr, *V2 = nullptr, *Q2 = nullptr, *G = nullptr;
  double *partials = nullptr, *acc = nullptr, *d_beta = nullptr;
  ~ct_tape() {
    for (float *b : bufs) (void)hipFree(b);
    (void)hipFree(partials);
    (void)hipFree(acc);
    (void)hipFree(d_beta);
  }
  int alloc(float **p, size_t count) {
    CT_TRY_HIP(hipMalloc(p, sizeof(float) * count));
    bufs.push_back(*p);
    return CT_OK;
  }
};

static int tape_alloc(ct_tape *t) {
  ct_solver *sv = t->sv;
  const size_t nb = sv->nb;
  const size_t nn = (size_t)sv->n * sv->n * nb, NM = (size_t)sv->N * sv->M * nb;
  for (int c = 0; c < t->n_ck; ++c) {
    float *u, *vb1, *vb2;
    CT_TRY(t->alloc(&u, nn));
    CT_TRY(t->alloc(&vb1, NM));
    CT_TRY(t->alloc(&vb2, 2 * nn));
    t->ck.push_back(u);
    t->ck.push_back(vb1);
    t->ck.push_back(vb2);
  }
  CT_TRY(t->alloc(&t->q1s, NM * t->every));
  CT_TRY(t->alloc(&t->q2s, 2 * nn * t->every));
  CT_TRY(t->alloc(&t->U, nn));
  CT_TRY(t->alloc(&t->Utot, nn));
  CT_TRY(t->alloc(&t->X, nn));
  CT_TRY(t->alloc(&t->V1, NM));
  CT_TRY(t->alloc(&t->P, NM));
  CT_TRY(t->alloc(&t->Q1, NM));
  CT_TRY(t->alloc(&t->bbar, NM));
  CT_TRY(t->alloc(&t->V2, 2 * nn));
  CT_TRY(t->alloc(&t->Q2, 2 * nn));
  CT_TRY(t->alloc(&t->G, 2 * nn));
  CT_TRY_HIP(hipMalloc(&t->partials, sizeof(double) * tv_reverse_partials(sv->n, sv->nb)));
  CT_TRY_HIP(hipMalloc(&t->acc, sizeof(double) * nb));
  CT_TRY_HIP(hipMalloc(&t->d_beta, sizeof(double)));
  return CT_OK;
}

static int copy_state(ct_solver *sv, float *u, float *vb1, float *vb2, bool out,
                      hipStream_t st) {
  const size_t nn = (size_t)sv->n * sv->n * sv->nb, NM = (size_t)sv->N * sv->M * sv->nb;
  const hipMemcpyKind kd = hipMemcpyDeviceToDevice;
  if (out) {
    CT_TRY_HIP(hipMemcpyAsync(u, sv->u, sizeof(float) * nn, kd, st));
    CT_TRY_HIP(hipMemcpyAsync(vb1, sv->vb1, sizeof(float) * NM, kd, st));
    CT_TRY_HIP(hipMemcpyAsync(vb2, sv->vb2, sizeof(float) * 2 * nn, kd, st));
  } else {
    CT_TRY_HIP(hipMemcpyAsync(sv->u, u, sizeof(float) * nn, kd, st));
    CT_TRY_HIP(hipMemcpyAsync(sv->vb1, vb1, sizeof(float) * NM, kd, st));
    CT_TRY_HIP(hipMemcpyAsync(sv->vb2, vb2, sizeof(float) * 2 * nn, kd, st));
  }
  return CT_OK;
}

extern "C" {

int ct_unrolled_forward(ct_solver *sv, int32_t K, int32_t every, ct_tape **out, ct_stream s) {
  clear_error();
  if (!sv || !out || K < 1 || every < 1) {
    set_error("ct_unrolled_forward: need a solver, K >= 1 and every >= 1");
    return CT_E_INVALID;
  }
  if (sv->ubar || sv->method != CT_METHOD_PDRQS1 || sv->fit != CT_FIT_STANDARD) {
    set_error("ct_unrolled_forward: the reverse sweep is for PDRQS1 without u >= 0");
    return CT_E_UNSUPPORTED;
  }
  *out = nullptr;
  hipStream_t st = S(s);
  std::unique_ptr<ct_tape> t(new (std::nothrow) ct_tape());
  if (!t) return CT_E_DEVICE;
  t->sv = sv;
  t->K = K;
  t->every = std::min(every, K);
  t->n_ck = (K + t->every - 1) / t->every;
  CT_TRY(tape_alloc(t.get()));
  CT_TRY(solver_zero_state(sv, st));
  ct_solver *one[1] = {sv};
  for (int c = 0; c < t->n_ck; ++c) {
    CT_TRY(copy_state(sv, t->ck[3 * c], t->ck[3 * c + 1], t->ck[3 * c + 2], true, st));
    const int k = std::min(t->every, K - c * t->every);
    CT_TRY(multi_step(one, 1, k, st, &sv->cap_stream, sv->gexec, sv->gexec_u));
  }
  t->iters_after = sv->iters;
  CT_TRY_HIP(hipStreamSynchronize(st));
  *out = t.release();
  return CT_OK;
}

int ct_unrolled_backward(ct_tape *t, const float *gbar, float *grad_u0, double *grad_lambda,
                         ct_stream s) {
  clear_error();
  if (!t || !gbar) {
    set_error("ct_unrolled_backward: null argument");
    return CT_E_INVALID;
  }
  ct_solver *sv = t->sv;
  if (sv->iters != t->iters_after) {
    set_error("ct_unrolled_backward: the solver was stepped after the forward pass");
    return CT_E_STATE;
  }
  hipStream_t st = S(s);
  ct_plan *p = sv->plan;
  const int n = sv->n, N = sv->N, M = sv->M, nb = sv->nb;
  const size_t nn = (size_t)n * n * nb, NM = (size_t)N * M * nb;
  const float sig = (float)sv->sigma, st_ = (float)(sv->sigma * sv->tau);
  const float inv_h = (float)(1.0 / p->g.h);
  const float rho = (float)(sv->lam_t / sv->tau);
  CT_TRY_HIP(hipMemcpyAsync(t->U, gbar, sizeof(float) * nn, hipMemcpyDeviceToDevice, st));
  CT_TRY_HIP(hipMemsetAsync(t->P, 0, sizeof(float) * NM, st));
  CT_TRY_HIP(hipMemsetAsync(t->V1, 0, sizeof(float) * NM, st));
  CT_TRY_HIP(hipMemsetAsync(t->bbar, 0, sizeof(float) * NM, st));
  CT_TRY_HIP(hipMemsetAsync(t->V2, 0, sizeof(float) * 2 * nn, st));
  CT_TRY_HIP(hipMemsetAsync(t->acc, 0, sizeof(double) * nb, st));
  for (int c = t->n_ck - 1; c >= 0; --c) {
    const int k0 = c * t->every;
    const int cnt = std::min(t->every, t->K - k0);
    // recompute the segment from its checkpoint, keeping the resolvent inputs
    CT_TRY(copy_state(sv, t->ck[3 * c], t->ck[3 * c + 1], t->ck[3 * c + 2], false, st));
    {
      const SinoEpi ep{(float)(1.0 / sv->beta), sig, sv->target, sv->mask, sv->vb1, sv->s1,
                       nullptr, nullptr, 1};
      CT_TRY(launch_radon_fwd(sv->fwd, sv->u, nullptr, st, &ep, nb));
      CT_TRY(launch_tv_update(n, inv_h, sv->u, st_, 0.0f, sv->vb2, sv->s2, nullptr, 1, st, nb));
    }
    for (int i = 0; i < cnt; ++i)
      CT_TRY(solver_iter(sv, 0, st, nullptr, t->q1s + i * NM, t->q2s + i * 2 * nn));
    for (int i = cnt - 1; i >= 0; --i) {
      CT_TRY(launch_sino_reverse(N, M, nb, sig, t->V1, t->q1s + i * NM, sv->target, sv->mask,
                                 t->P, t->Q1, t->bbar, st));
      CT_TRY(launch_tv_reverse(n, nb, st_, rho, t->V2, t->q2s + i * 2 * nn, t->Q2, t->G,
                               t->partials, t->acc, st));
      // Utot = U + A^* P - div G
      CT_TRY(launch_radon_adj(p, t->P, t->G, (float)(1.0 / sv->beta), -1.0f, t->Utot, st, nb,
                              sv->bp_part, sv->bp_S, sv->bp_kern, t->U));
      CT_TRY(launch_apply_mult(&sv->pc, sv->pc.d_mult, t->Utot, nullptr, t->X, st, nb,
                               sv->spec));
      SinoEpi ep{(float)(1.0 / sv->beta), sig, nullptr, nullptr, t->Q1, t->V1, t->P, nullptr,
                 3};
      CT_TRY(launch_radon_fwd(sv->fwd, t->X, nullptr, st, &ep, nb));
      CT_TRY(launch_img_tail(n, nb, st_, inv_h, t->X, t->Q2, t->Utot, t->U, t->V2, st));
    }
  }
  t->iters_after = sv->iters;
  if (grad_u0) {
    const double beta = sv->beta;
    CT_TRY_HIP(hipMemcpyAsync(t->d_beta, &beta, sizeof(double), hipMemcpyHostToDevice, st));
    CT_TRY(launch_scale_by_inv(t->bbar, (int64_t)NM, t->d_beta, grad_u0, st));
  }
  std::vector<double> acc(nb);
  CT_TRY_HIP(hipMemcpyAsync(acc.data(), t->acc, sizeof(double) * nb, hipMemcpyDeviceToHost, st));
  CT_TRY_HIP(hipStreamSynchronize(st));
  if (grad_lambda)
    for (int b = 0; b < nb; ++b) grad_lambda[b] = acc[b] / (sv->beta * sv->beta * sv->tau);
  return CT_OK;
}

int ct_tape_destroy(ct_tape *t) {
  clear_error();
  delete t;
  return CT_OK;
}

}  // extern "C"
