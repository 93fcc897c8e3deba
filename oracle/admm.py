"""ADMM with an inner preconditioned conjugate-gradient solve (thesis §4.6)
and the isotropic soft thresholding of its z-update (lemma of §4.6), for the
unconstrained problem (P_h).  Test infrastructure only (see the package
header).

On the normalized problem of §5.1 (A = R_h / beta, b = u0 / beta,
lambda~ = lambda / beta^2; the same Setup as PDRQS1) the splitting is
  min_{u, z} f(z)  s.t.  z = K u,   K = [A; nabla_h],
  f(w, v) = 1/2 ||w - b||^2 + lambda~ ||v||_1   (isotropic),
with the augmented Lagrangian weighted by Lambda = diag(I, tau I):
  L(u, z, eta) = f(z) + mu/2 ||z - K u - eta||_Lambda^2.
One ADMM iteration from (u, z, eta):
  u-step : approximately solve H u = A^*(z_w - eta_w) - tau^2 div(z_v - eta_v),
           H = A^* A - tau^2 div nabla  (= K^T Lambda^2 K),
           by `cg_steps` PCG steps started from the current u;
  z-step : w = (b + mu (A u + eta_w)) / (1 + mu),
           v = soft(nabla u + eta_v, lambda~ / (mu tau^2));
  eta    : eta <- eta - (z - K u).
Readings:
  * the z_v penalty: the thesis' "mu nu / 2" with nu = tau^2, the weight that
    Lambda gives the gradient block (K^T Lambda^2 K above has the same tau^2);
  * the multiplier update: the printed eta <- eta - mu (z - K u) has a factor
    mu that the derivation (eta = -Lambda^-2 gamma / mu, gamma ascending by
    mu Lambda^2 (z - K u)) does not give; the iteration uses the scaled form
    eta <- eta - (z - K u), which agrees with the printed one at mu = 1;
  * the preconditioner of the PCG is the inverse-norm one of §4.3.1 for
    alpha = 1, beta = tau^2: M^{-1} = F^{-1} rho_eps / (c + tau^2 lambda_Delta
    rho_eps) F, with the same c as PDRQS1 (the thesis allows any of its
    preconditioners here);
  * PCG from the current u (warm start), restarted in every ADMM iteration
    (its right-hand side changes); a step whose search direction has
    p.Hp = 0 (zero residual) moves nothing (alpha = 0), and beta = 0 when
    the previous r.z is 0;
  * initial values: u = 0, z = K u = 0, eta = 0.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import precond, tv
from .pdrq import Setup


def soft_threshold(q: np.ndarray, t: float) -> np.ndarray:
    """Pixelwise minimizer of 1/2 |x - q|^2 + t |x| for 2-vectors (lemma of
    §4.6): 0 where |q| <= t, else (1 - t/|q|) q."""
    nrm = np.sqrt(q[0] ** 2 + q[1] ** 2)
    scale = np.where(nrm > t, 1.0 - t / np.where(nrm > 0, nrm, 1.0), 0.0)
    return q * scale


def multiplier_admm(n: int, tau: float, c: float, eps: float) -> np.ndarray:
    """rho_eps / (c + tau^2 lambda_Delta rho_eps): the inverse-norm
    preconditioner of §4.3.1 for H = A^* A - tau^2 Delta_h."""
    r = precond.rho_eps(n, eps)
    return r / (c + tau * tau * precond.lap_symbol(n) * r)


def H(s: Setup, u: np.ndarray) -> np.ndarray:
    """H u = A^* A u - tau^2 div nabla u."""
    h = s.problem.geom.h
    tau = s.params.tau
    return s.At(s.A(u)) - tau * tau * tv.div(tv.grad(u, h), h)


def pcg(s: Setup, rhs: np.ndarray, u: np.ndarray, steps: int, mult: np.ndarray):
    """`steps` preconditioned conjugate-gradient steps on H u = rhs from u."""
    r = rhs - H(s, u)
    z = precond.apply_multiplier(r, mult)
    rz = float(np.sum(r * z))
    p = z.copy()
    for _ in range(steps):
        Hp = H(s, p)
        pHp = float(np.sum(p * Hp))
        alpha = rz / pHp if pHp > 0 else 0.0
        u = u + alpha * p
        r = r - alpha * Hp
        z = precond.apply_multiplier(r, mult)
        rz_new = float(np.sum(r * z))
        beta = rz_new / rz if rz > 0 else 0.0
        p = z + beta * p
        rz = rz_new
    return u


@dataclasses.dataclass
class State:
    u: np.ndarray
    zw: np.ndarray      # (N, M)
    zv: np.ndarray      # (2, n, n)
    ew: np.ndarray      # eta_w
    ev: np.ndarray      # eta_v


def zero_state(s: Setup) -> State:
    g = s.problem.geom
    return State(np.zeros((g.n, g.n)), np.zeros((g.n_angles, g.n_bins)),
                 np.zeros((2, g.n, g.n)), np.zeros((g.n_angles, g.n_bins)),
                 np.zeros((2, g.n, g.n)))


def step(s: Setup, st: State, cg_steps: int = 1, mu: float = 1.0) -> State:
    """One ADMM iteration (§4.6), in the order u-step, z-step, eta-update."""
    h = s.problem.geom.h
    tau = s.params.tau
    mult = multiplier_admm(s.problem.geom.n, tau, s.c, s.params.eps)
    rhs = s.At(st.zw - st.ew) - tau * tau * tv.div(st.zv - st.ev, h)
    u = pcg(s, rhs, st.u, cg_steps, mult)
    Au, gu = s.A(u), tv.grad(u, h)
    zw = (s.b + mu * (Au + st.ew)) / (1.0 + mu)
    zv = soft_threshold(gu + st.ev, s.lam_t / (mu * tau * tau))
    ew = st.ew - (zw - Au)
    ev = st.ev - (zv - gu)
    return State(u, zw, zv, ew, ev)


def run(s: Setup, iters: int, cg_steps: int = 1, mu: float = 1.0) -> State:
    st = zero_state(s)
    for _ in range(iters):
        st = step(s, st, cg_steps, mu)
    return st
