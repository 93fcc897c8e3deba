"""Algorithm CP (thesis §3.4), the unpreconditioned primal-dual method.

Applied to the normalized problem of §5.1 (A = R_h/beta, b, C~, lambda~),
K = [A; nabla_h], F = 0; with dual variables v (sinogram) and w (gradient
field), from u = bar u = v = w = 0:
  bar w = w + tau nabla bar u ;  bar v = v + tau A bar u
  w = bar w / max(1, |bar w| / lambda~)
  v = prox_sino(bar v, tau)
  u_new = u + sigma div w - sigma A^* v
  bar u = 2 u_new - u ;  u = u_new
It converges for sigma tau ||K||^2 < 1, i.e. sigma tau < 1/9 after the
normalization (||A|| <= 1, ||nabla_h||^2 < 8).  The tests use it as an
independent solver for the same minimizer as PDRQS1.
"""
from __future__ import annotations

import numpy as np

from . import prox, tv


def run(A, At, b, cb, mask, lam_t, n, iters, sigma, tau, h=1.0, resolvent=None):
    """Returns (u, v, w) after `iters` CP iterations; A/At act on (n, n) images.
    resolvent(q, step) replaces the standard data-term resolvent (variants)."""
    u = np.zeros((n, n))
    ub = np.zeros((n, n))
    v = np.zeros_like(np.asarray(b, dtype=np.float64))
    w = np.zeros((2, n, n))
    for _ in range(iters):
        wb = w + tau * tv.grad(ub, h)
        vb = v + tau * A(ub)
        w = prox.tv_project(wb, lam_t)
        v = (prox.prox_sino(vb, tau, b, cb, mask) if resolvent is None
             else resolvent(vb, tau))
        u_new = u + sigma * tv.div(w, h) - sigma * At(v)
        ub = 2.0 * u_new - u
        u = u_new
    return u, v, w
