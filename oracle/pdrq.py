"""Problem setup and Algorithm PDRQS1 (thesis §4.4, §5.1).

The problem (C_h) of §3.2:
  min_u  1/2 ||R_h u - u0||^2 on D\\D0  +  lambda ||nabla_h u||_1
         subject to (R_h u) >= C on the metal trace D0.
D0 empty gives the unconstrained problem (P_h).

Normalization (§5.1): the algorithm runs on A = R_h / beta with data
b = u0 / beta, bounds C / beta and weight lambda~ = lambda / beta^2, which has
the same minimizers.  Reading: beta is the power-iteration estimate of
||R_h|| rather than the crude lemma bound, so that ||A|| is close to 1.

PDRQS1 (§4.4, splitting PDRQ1 of the table of splittings: Q = f = S = g = 0,
K = [A; tau nabla_h]), one iteration from (u, vb1, vb2):
  u_tmp = -sigma ( A^*(vb1 + sigma A u) - tau div(vb2 + sigma tau nabla u) )
  u_new = u + M^{-1} u_tmp
  v1 = vb1 + sigma A u_new ;  v2 = vb2 + sigma tau nabla u_new
  y1 = prox_sino(2 v1 - vb1, sigma) ;  vb1 <- vb1 + y1 - v1
  w  = tv_project(2 v2 - vb2, lambda~/tau) ;  vb2 <- vb2 + w - v2
  u <- u_new
As the thesis remarks in §4.4, A u and nabla u of the previous iterate can be
kept, so that A and A^* are applied once per iteration; the state carries
r = A u and g = nabla u for that purpose.  Initial values (unspecified in the
thesis): all zero.  Defaults for the step parameters (unspecified in the
thesis for PDRQ): sigma = 1, tau = 1/sqrt(8) on the normalized problem,
eps = 0.3, c = 1.1 * lambda_max.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

from . import power, precond, prox, radon, tv
from .geometry import Geometry


@dataclasses.dataclass
class Problem:
    geom: Geometry
    u0: np.ndarray          # (N, M) measured sinogram
    mask: np.ndarray        # (N, M) bool, metal trace D0
    bound: np.ndarray       # (N, M) lower bounds C (used on D0 only)
    lam: float              # lambda of (C_h), unnormalized


@dataclasses.dataclass
class Params:
    sigma: float = 1.0
    tau: float = 1.0 / math.sqrt(8.0)
    eps: float = 0.3
    c_safety: float = 1.1
    power_iters: int = 30


@dataclasses.dataclass
class Setup:
    """Normalized problem: A = R_h/beta, b = u0/beta, cb = C/beta, lam_t = lambda/beta^2."""
    problem: Problem
    params: Params
    beta: float
    c: float
    b: np.ndarray
    cb: np.ndarray
    lam_t: float
    mult: np.ndarray
    fwd: object = None      # R_h (defaults to radon.radon_fwd on the geometry)
    adj: object = None      # R_h^* (defaults to radon.radon_adj)
    fit: str = "standard"   # data term variant of §3.5 (see sino_resolvent)
    weight: object = None   # per-bin weights of the weighted fit (default 1)

    def A(self, u):
        f = self.fwd or (lambda x: radon.radon_fwd(self.problem.geom, x))
        return f(u) / self.beta

    def At(self, v):
        f = self.adj or (lambda y: radon.radon_adj(self.problem.geom, y))
        return f(v) / self.beta


def setup(problem: Problem, params: Params, start_norm: np.ndarray | None = None,
          start_precond: np.ndarray | None = None, beta: float | None = None,
          c: float | None = None, fwd=None, adj=None, kind: str = "invnorm") -> Setup:
    """Normalization (§5.1) and preconditioner constant (§4.3.1, §4.3.2).

    beta and c are estimated by power iteration from the given start images
    unless passed explicitly.  fwd/adj replace R_h/R_h^* (e.g. by an explicit
    matrix on tiny problems); by default the radon module's pair is used.
    kind selects the preconditioner of PDRQS1: "invnorm" (§4.3.1: c scales the
    inverse-norm part), "impulse" (§4.3.2: c scales M_K, the deconvolution
    by the impulse response of A^* A plus the periodic Laplacian) or
    "circulant" (§4.3.3: the same on the vectorized image, with the 1-D DFT;
    mult then holds the length-n^2 symbol, applied by apply_precond).
    """
    g = problem.geom
    fwd = fwd or (lambda u: radon.radon_fwd(g, u))
    adj = adj or (lambda v: radon.radon_adj(g, v))
    if beta is None:
        beta = power.radon_norm(fwd, adj, start_norm, params.power_iters)
    A = lambda u: fwd(u) / beta
    At = lambda v: adj(v) / beta
    if kind == "impulse":
        sig, tau = params.sigma, params.tau
        khat = precond.kernel_symbol(precond.impulse_kernel(A, At, g.n))
        fK = precond.impulse_full_symbol(khat, sig * sig, (sig * tau) ** 2)
        if not np.all(fK > 0):
            raise ValueError("impulse-response preconditioner: F(K) is not positive")
        if c is None:
            c = params.c_safety * power.impulse_constant_eig(
                A, At, fK, sig * sig, (sig * tau) ** 2, g.h, start_precond, params.power_iters)
        mult = precond.impulse_multiplier(fK, c)
    elif kind == "circulant":
        sig, tau = params.sigma, params.tau
        fK = precond.circulant_full_symbol(precond.circulant_kernel(A, At, g.n), sig * sig,
                                           (sig * tau) ** 2)
        if not np.all(fK > 0):
            raise ValueError("circulant preconditioner: F_L(K) is not positive")
        if c is None:
            c = params.c_safety * power.circulant_constant_eig(
                A, At, fK, sig * sig, (sig * tau) ** 2, g.h, start_precond, params.power_iters)
        mult = 1.0 / (c * fK)
    else:
        if c is None:
            lmax = power.precond_constant_eig(A, At, start_precond, params.eps,
                                              params.power_iters)
            c = params.c_safety * lmax
        mult = precond.multiplier(g.n, params.sigma, params.tau, c, params.eps)
    return Setup(problem, params, float(beta), float(c),
                 np.asarray(problem.u0, dtype=np.float64) / beta,
                 np.asarray(problem.bound, dtype=np.float64) / beta,
                 problem.lam / beta ** 2, mult, fwd, adj)


def apply_precond(s: Setup, y: np.ndarray) -> np.ndarray:
    """M^{-1} y: a 2-D Fourier multiplier, or (circulant preconditioner, a
    length-n^2 symbol) the 1-D one on the vectorized image."""
    if s.mult.ndim == 1:
        return precond.apply_circulant(y, s.mult)
    return precond.apply_multiplier(y, s.mult)


def sino_resolvent(s: Setup, q: np.ndarray, step: float) -> np.ndarray:
    """Resolvent of the data term's conjugate at q, for the variants of §3.5:
    standard (fit off D0, C~ <= A u on D0), weighted (weights on the fit),
    ignore (no term on D0), everywhere (fit on all bins plus C~ <= A u on D0),
    hard (A u = b off D0, C~ <= A u on D0)."""
    mask = s.problem.mask
    if s.fit == "standard":
        return prox.prox_sino(q, step, s.b, s.cb, mask)
    if s.fit == "weighted":
        w = np.ones_like(s.b) if s.weight is None else np.asarray(s.weight, dtype=np.float64)
        return prox.prox_sino_weighted(q, step, s.b, w, s.cb, mask)
    if s.fit == "ignore":
        return prox.prox_sino_ignore(q, step, s.b, mask)
    if s.fit == "everywhere":
        return prox.prox_sino_fit_everywhere(q, step, s.b, s.cb, mask)
    if s.fit == "hard":
        return prox.prox_sino_hard(q, step, s.b, s.cb, mask)
    raise ValueError(f"unknown data term variant {s.fit!r}")


@dataclasses.dataclass
class State:
    u: np.ndarray      # (n, n)
    vb1: np.ndarray    # (N, M)  bar v_1
    vb2: np.ndarray    # (2, n, n) bar v_2
    r: np.ndarray      # A u (cached)
    g: np.ndarray      # nabla_h u (cached)

    def copy(self):
        return State(self.u.copy(), self.vb1.copy(), self.vb2.copy(), self.r.copy(), self.g.copy())


def zero_state(s: Setup) -> State:
    g = s.problem.geom
    n, N, M = g.n, g.n_angles, g.n_bins
    return State(np.zeros((n, n)), np.zeros((N, M)), np.zeros((2, n, n)),
                 np.zeros((N, M)), np.zeros((2, n, n)))


def state_from(s: Setup, u, vb1, vb2) -> State:
    """A state with its caches recomputed from (u, vb1, vb2)."""
    u = np.asarray(u, dtype=np.float64)
    return State(u.copy(), np.asarray(vb1, dtype=np.float64).copy(),
                 np.asarray(vb2, dtype=np.float64).copy(), s.A(u), tv.grad(u, s.problem.geom.h))


def step(s: Setup, st: State, return_dual: bool = False):
    """One PDRQS1 iteration (§4.4).  Returns the new state, and with
    return_dual also (y1, w), the resolvent outputs of this iteration."""
    sig, tau = s.params.sigma, s.params.tau
    h = s.problem.geom.h
    s1 = st.vb1 + sig * st.r
    s2 = st.vb2 + sig * tau * st.g
    u_tmp = -sig * (s.At(s1) - tau * tv.div(s2, h))
    u_new = st.u + apply_precond(s, u_tmp)
    r_new = s.A(u_new)
    g_new = tv.grad(u_new, h)
    v1 = st.vb1 + sig * r_new
    v2 = st.vb2 + sig * tau * g_new
    y1 = sino_resolvent(s, 2.0 * v1 - st.vb1, sig)
    vb1 = st.vb1 + y1 - v1
    w = prox.tv_project(2.0 * v2 - st.vb2, s.lam_t / tau)
    vb2 = st.vb2 + w - v2
    new = State(u_new, vb1, vb2, r_new, g_new)
    if return_dual:
        return new, y1, w
    return new


def run(s: Setup, iters: int, st: State | None = None, record_every: int = 0):
    """iters PDRQS1 iterations from st (zero state by default).

    With record_every > 0, also returns the gap records (oracle.gap.record)
    taken after every record_every-th iteration.
    """
    from . import gap
    st = zero_state(s) if st is None else st
    records = []
    for k in range(iters):
        want = record_every > 0 and (k + 1) % record_every == 0
        if want:
            prev = st.u
            st, y1, w = step(s, st, return_dual=True)
            records.append(gap.record(s, st.u, y1, w, prev))
        else:
            st = step(s, st)
    return (st, records) if record_every > 0 else st


# ---------------------------------------------------------------------------
# Variant with u >= 0 (§4.5): PDRQS1 with the extra state bar u and the
# non-negativity resolvent; preconditioner id + c sigma^2 tilde M - (sigma tau)^2 Delta_p.

@dataclasses.dataclass
class StateNonneg:
    u: np.ndarray
    ub: np.ndarray
    vb1: np.ndarray
    vb2: np.ndarray
    r: np.ndarray
    g: np.ndarray


def zero_state_nonneg(s: Setup) -> StateNonneg:
    z = zero_state(s)
    return StateNonneg(z.u, np.zeros_like(z.u), z.vb1, z.vb2, z.r, z.g)


def step_nonneg(s: Setup, st: StateNonneg) -> StateNonneg:
    """One iteration of the u >= 0 variant of PDRQS1 (§4.5)."""
    sig, tau = s.params.sigma, s.params.tau
    h = s.problem.geom.h
    mult = precond.multiplier_nonneg(s.problem.geom.n, sig, tau, s.c, s.params.eps)
    s1 = st.vb1 + sig * st.r
    s2 = st.vb2 + sig * tau * st.g
    u_tmp = st.ub - st.u - sig * (s.At(s1) - tau * tv.div(s2, h))
    u_new = st.u + precond.apply_multiplier(u_tmp, mult)
    r_new = s.A(u_new)
    g_new = tv.grad(u_new, h)
    v1 = st.vb1 + sig * r_new
    v2 = st.vb2 + sig * tau * g_new
    y1 = sino_resolvent(s, 2.0 * v1 - st.vb1, sig)
    vb1 = st.vb1 + y1 - v1
    w = prox.tv_project(2.0 * v2 - st.vb2, s.lam_t / tau)
    vb2 = st.vb2 + w - v2
    ub = st.ub + prox.prox_nonneg(2.0 * u_new - st.ub) - u_new
    return StateNonneg(u_new, ub, vb1, vb2, r_new, g_new)
