"""Algorithm PDRQS2 (thesis §4.2, §4.3.1) and the Richardson choice of M (§4.3)
for comparison with PDRQS1 and Algorithm CP.  Test infrastructure only (see
the package header).

PDRQS2 treats the unconstrained problem (P_h) with the data term kept in the
primal as the linear-quadratic part Q = A^* A, f = -A^* b, and K = tau nabla_h
(G^* the indicator of the ball of radius lambda~/tau).  With the normalization
of §5.1 (A = R_h/beta, b = u0/beta, lambda~ = lambda/beta^2), from (u, vb):
  u_tmp = sigma tau div vb + sigma A^*(b - A u) + (sigma tau)^2 div nabla u
  u_new = u + M^{-1} u_tmp,   M^{-1}: rho_eps / (sigma c + (sigma tau)^2 lambda_Delta rho_eps)
  v     = vb + sigma tau nabla u_new
  w     = tv_project(2 v - vb, lambda~/tau);  vb <- vb + w - v
Reading: the printed Laplacian term is -(sigma tau)^2 laph u with
laph = -div nabla; with T = sigma Q + sigma^2 K^* K this is
+(sigma tau)^2 div nabla u, which the iteration above uses.  c is the same
constant as for PDRQS1: c tilde M >= A^* A.

Richardson (§4.3): M = m id with m > ||T||.  For PDRQS1,
T = sigma^2 A^* A - (sigma tau)^2 Delta_h and ||T|| <= sigma^2 ||A||^2 + 8 (sigma tau)^2
(h = 1); the reading takes m = 1.1 (sigma^2 + 8 (sigma tau)^2) with ||A|| = 1
after the normalization.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import precond, prox, tv
from .pdrq import Setup


def multiplier2(n: int, sigma: float, tau: float, c: float, eps: float) -> np.ndarray:
    """rho_eps / (sigma c + (sigma tau)^2 lambda_Delta rho_eps)  (PDRQS2)."""
    r = precond.rho_eps(n, eps)
    return r / (sigma * c + (sigma * tau) ** 2 * precond.lap_symbol(n) * r)


def richardson_m(sigma: float, tau: float, h: float = 1.0) -> float:
    return 1.1 * (sigma * sigma + 8.0 * (sigma * tau) ** 2 / (h * h))


@dataclasses.dataclass
class State2:
    u: np.ndarray
    vb: np.ndarray   # (2, n, n)


def zero_state2(s: Setup) -> State2:
    n = s.problem.geom.n
    return State2(np.zeros((n, n)), np.zeros((2, n, n)))


def step2(s: Setup, st: State2) -> State2:
    """One PDRQS2 iteration (requires D0 empty)."""
    sig, tau = s.params.sigma, s.params.tau
    h = s.problem.geom.h
    mult = multiplier2(s.problem.geom.n, sig, tau, s.c, s.params.eps)
    u_tmp = (sig * tau * tv.div(st.vb, h) + sig * s.At(s.b - s.A(st.u))
             + (sig * tau) ** 2 * tv.div(tv.grad(st.u, h), h))
    u_new = st.u + precond.apply_multiplier(u_tmp, mult)
    v = st.vb + sig * tau * tv.grad(u_new, h)
    w = prox.tv_project(2.0 * v - st.vb, s.lam_t / tau)
    return State2(u_new, st.vb + w - v)


def richardson_setup(s: Setup) -> Setup:
    """The same normalized problem with M = m id in PDRQS1 (pdrq.step then
    computes u_new = u + u_tmp / m)."""
    n = s.problem.geom.n
    m = richardson_m(s.params.sigma, s.params.tau, s.problem.geom.h)
    return dataclasses.replace(s, mult=np.full((n, n), 1.0 / m))


def objective(s: Setup, u: np.ndarray):
    """(1/2 sum_{D\\D0} (R_h u - u0)^2, lambda TV(u), max_{D0} (C - R_h u)_+) in
    the problem's own (unnormalized) units."""
    g = s.problem.geom
    r = s.A(u) * s.beta
    mask = s.problem.mask
    fit = 0.5 * float(np.sum(np.where(mask, 0.0, (r - s.problem.u0) ** 2)))
    reg = s.problem.lam * tv.tv(u, g.h)
    viol = float(np.max(np.where(mask, s.problem.bound - r, 0.0), initial=0.0))
    return fit, reg, max(viol, 0.0)
