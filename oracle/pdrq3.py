"""Splitting PDRQ3 of the thesis' table of splittings (§4.4): the quadratic
part of the data term moved into the dual linear-quadratic part.  Test
infrastructure only (see the package header).

With Q = f = 0, K = [A; tau nabla_h], S = diag(chi_Omega, 0) and
g = (b chi_Omega, 0) (Omega = D \\ D0), the remaining G~* is the constraint
on D0 (its conjugate) and the TV ball.  The thesis derives the linear-
quadratic PDRQ for S = nu id; with the diagonal S here the same derivation
holds entrywise, D = (mu + sigma S)^{-1} taking 1/(1 + sigma) on Omega's bins
and 1 on D0 and on the gradient (mu = 1).  One iteration from (u, vb1, vb2):
  s1 = D1 (vb1 + sigma (A u - g1)),  s2 = vb2 + sigma tau nabla u
  u_new = u + M^{-1}( -sigma (A^* s1 - tau div s2) )
  Omega:  v1 = (vb1 + sigma (A u_new - b)) / (1 + sigma);  vb1 <- v1
          (the resolvent of G~* there is the identity)
  D0:     v1 = vb1 + sigma A u_new;  y = min(2 v1 - vb1 - sigma C~, 0);
          vb1 <- vb1 + y - v1
  gradient: as PDRQS1 (v2 = vb2 + sigma tau nabla u_new, w = projection of
          2 v2 - vb2 on the ball of radius lambda~/tau, vb2 <- vb2 + w - v2).
Readings:
  * the entrywise extension of the S = nu id derivation (the table lists
    PDRQ3 with this diagonal S without restating the iteration), with the
    dual linear term g inside the u-step's argument, -sigma K^* D (vb +
    sigma (K u - g)): the printed b^k carries "- sigma f" inside K^*(...),
    where only the dual g fits; this is the form whose fixed points satisfy
    0 in S v + g - K u + dG~*(v) and K^* v = 0;
  * the resolvent on D0: the printed min(v/(1 + sigma C), 0) does not follow
    from G~*; the conjugate of the constraint on D0 is the same as in PDRQS1,
    whose resolvent is min(q - sigma C~, 0);
  * M: PDRQS1's preconditioner, valid because T~ = sigma^2 K^* D K <=
    sigma^2 K^* K.
"""
from __future__ import annotations

import numpy as np

from . import precond, prox, tv
from .pdrq import Setup, State, apply_precond


def step3(s: Setup, st: State) -> State:
    sig, tau = s.params.sigma, s.params.tau
    h = s.problem.geom.h
    mask = s.problem.mask
    # D (vb + sigma (K u - g)) of the sinogram block: g = b on Omega
    s1 = np.where(mask, st.vb1 + sig * st.r, (st.vb1 + sig * (st.r - s.b)) / (1.0 + sig))
    s2 = st.vb2 + sig * tau * st.g
    u_new = st.u + apply_precond(s, -sig * (s.At(s1) - tau * tv.div(s2, h)))
    r = s.A(u_new)
    g = tv.grad(u_new, h)
    v1_off = (st.vb1 + sig * (r - s.b)) / (1.0 + sig)
    v1_on = st.vb1 + sig * r
    y_on = np.minimum(2.0 * v1_on - st.vb1 - sig * s.cb, 0.0)
    vb1 = np.where(mask, st.vb1 + y_on - v1_on, v1_off)
    v2 = st.vb2 + sig * tau * g
    w = prox.tv_project(2.0 * v2 - st.vb2, s.lam_t / tau)
    return State(u_new, vb1, st.vb2 + w - v2, r, g)


def run3(s: Setup, iters: int, st: State | None = None) -> State:
    from .pdrq import zero_state
    st = st or zero_state(s)
    for _ in range(iters):
        st = step3(s, st)
    return st
