"""Reverse-mode derivative of K unrolled PDRQS1 iterations (thesis §4.4).

Test infrastructure only (see the package header).

The map from the data u0 and the weight lambda to the K-th iterate u_K is a
composition of K iterations of PDRQS1, each a linear map (A, A^*, nabla, div,
M^{-1}) followed by the two pointwise resolvents.  Both resolvents are
piecewise smooth, so u_K is differentiable almost everywhere and its
derivative is the chain rule through every step.  This module writes that
chain rule out in plain FP64, one iteration at a time, in the order the steps
are taken, for a scalar loss L(u_K) with gradient gbar = dL/du_K.

One iteration from (u, vb1, vb2), with A = R_h/beta, b = u0/beta,
rho = lambda~/tau = lambda/(beta^2 tau):
  s1 = vb1 + sigma A u,  s2 = vb2 + sigma tau nabla u
  u' = u + M^{-1}(-sigma A^* s1 + sigma tau div s2)
  q1 = vb1 + 2 sigma A u'          (= 2 v1 - vb1)
  y1 = P1(q1; b):  (q1 - sigma b)/(1 + sigma) off D0,  min(q1 - sigma C~, 0) on D0
  vb1' = y1 - sigma A u'           (= vb1 + y1 - v1)
  q2 = vb2 + 2 sigma tau nabla u'
  w = P2(q2; rho) = q2 min(1, rho/|q2|)  pixelwise
  vb2' = w - sigma tau nabla u'

Jacobians of the resolvents (where they are differentiable):
  dP1/dq1 = 1/(1+sigma) off D0; [q1 - sigma C~ < 0] on D0;  dP1/db = -sigma/(1+sigma) off D0
  dP2/dq2 = I where |q2| <= rho, else (rho/|q2|)(I - qhat qhat^T);  dP2/drho = [|q2| > rho] qhat
M^{-1} is real and symmetric (a real even multiplier in the Fourier domain),
A^* is the transpose of A and -div is the transpose of nabla.
"""
from __future__ import annotations

import numpy as np

from . import precond, tv
from .pdrq import Setup, State, step, zero_state


def forward(s: Setup, K: int) -> list[State]:
    """States 0..K of PDRQS1 from the zero state."""
    states = [zero_state(s)]
    for _ in range(K):
        states.append(step(s, states[-1]))
    return states


def _resolvent_inputs(s: Setup, st: State, nxt: State):
    """q1 and q2 of the iteration st -> nxt (recomputed from the two states)."""
    sig, tau = s.params.sigma, s.params.tau
    q1 = st.vb1 + 2.0 * sig * nxt.r
    q2 = st.vb2 + 2.0 * sig * tau * nxt.g
    return q1, q2


def backward(s: Setup, states: list[State], gbar: np.ndarray):
    """dL/du0 (N, M) and dL/dlambda for L with dL/du_K = gbar."""
    sig, tau = s.params.sigma, s.params.tau
    h = s.problem.geom.h
    mask = s.problem.mask
    rho = s.lam_t / tau
    K = len(states) - 1
    # adjoints of the state after the current iteration
    U = np.array(gbar, dtype=np.float64)
    V1 = np.zeros_like(states[0].vb1)
    V2 = np.zeros_like(states[0].vb2)
    bbar = np.zeros_like(V1)
    rhobar = 0.0
    for k in range(K - 1, -1, -1):
        st, nxt = states[k], states[k + 1]
        q1, q2 = _resolvent_inputs(s, st, nxt)
        # vb1' = y1 - sigma A u',  y1 = P1(q1; b)
        Y1 = V1
        d1 = np.where(mask, (q1 - sig * s.cb < 0.0).astype(np.float64), 1.0 / (1.0 + sig))
        Q1 = d1 * Y1
        bbar += np.where(mask, 0.0, -sig / (1.0 + sig) * Y1)
        R_new = -sig * V1 + 2.0 * sig * Q1          # adjoint of A u'
        # vb2' = w - sigma tau nabla u',  w = P2(q2; rho)
        W = V2
        nq = np.sqrt(q2[0] ** 2 + q2[1] ** 2)
        out = nq > rho
        safe = np.where(nq > 0, nq, 1.0)
        qh = q2 / safe
        qh_dot_w = qh[0] * W[0] + qh[1] * W[1]
        Q2 = np.where(out, (rho / safe) * (W - qh * qh_dot_w), W)
        rhobar += float(np.sum(np.where(out, qh_dot_w, 0.0)))
        G_new = -sig * tau * V2 + 2.0 * sig * tau * Q2   # adjoint of nabla u'
        # u' = u + M^{-1} u_tmp; u' also feeds q1, q2, vb1', vb2' through A u', nabla u'
        U_new = U + s.At(R_new) - tv.div(G_new, h)
        Utmp = precond.apply_multiplier(U_new, s.mult)
        # u_tmp = -sigma A^* s1 + sigma tau div s2
        S1 = -sig * s.A(Utmp)
        S2 = -sig * tau * tv.grad(Utmp, h)
        # s1 = vb1 + sigma A u, s2 = vb2 + sigma tau nabla u
        U = U_new + sig * s.At(S1) - sig * tau * tv.div(S2, h)
        V1 = Q1 + S1
        V2 = Q2 + S2
    du0 = bbar / s.beta
    dlam = rhobar / (s.beta ** 2 * tau)
    return du0, dlam


def mse_loss(u: np.ndarray, ref: np.ndarray):
    """L = mean (u - ref)^2 and its gradient."""
    d = u - ref
    return float(np.mean(d * d)), 2.0 * d / d.size
