"""Primal-dual record in FP64 (a reading; the thesis defines no gap).

The thesis plots objective values relative to the smallest attained one and
states no gap.  With F = 0 the Fenchel dual of (C_h) (§3.3, duality of
§1.3) is finite only where K^* y = 0, so the textbook gap is infinite off the
solution.  The record computed here, in normalized units (§5.1) and with
y = (y1, w) the resolvent outputs of the last PDRQS1 iteration, is:

  P(u)   = 1/2 sum_{D\\D0} (A u - b)^2 + lambda~ sum |nabla u|   (indicator dropped)
  G*(y)  = sum_{D\\D0} (1/2 y1^2 + y1 b) + sum_{D0} y1 C~         (§3.3 conjugates;
           finite since y1 <= 0 on D0 and |w| <= lambda~/tau by construction)
  gap    = P(u) + G*(y)
  rho_D  = ||A^* y1 - tau div w||  (= ||K^* y|| with K = [A; tau nabla])
  V      = max_{D0} (C~ - A u)_+     (constraint violation)
  du     = ||u_new - u_prev||

At a saddle point gap = rho_D = V = 0.  The Fenchel-Young inequality gives
gap - <u, K^* y> >= 0 whenever A u >= C~ on D0.
"""
from __future__ import annotations

import numpy as np

from . import tv


def record(s, u: np.ndarray, y1: np.ndarray, w: np.ndarray,
           u_prev: np.ndarray | None = None) -> np.ndarray:
    """(P, G*, gap, rho_D, V, du) as float64 for setup s (oracle.pdrq.Setup)."""
    h = s.problem.geom.h
    tau = s.params.tau
    mask = s.problem.mask
    off = ~mask
    Au = s.A(u)
    gu = tv.grad(u, h)
    P = 0.5 * np.sum(((Au - s.b) ** 2)[off]) + s.lam_t * np.sum(np.sqrt(gu[0] ** 2 + gu[1] ** 2))
    Gs = np.sum((0.5 * y1 ** 2 + y1 * s.b)[off]) + np.sum((y1 * s.cb)[mask])
    Kty = s.At(y1) - tau * tv.div(w, h)
    rho = np.sqrt(np.sum(Kty ** 2))
    V = float(np.max(np.maximum(s.cb - Au, 0.0)[mask])) if mask.any() else 0.0
    du = float(np.sqrt(np.sum((u - u_prev) ** 2))) if u_prev is not None else 0.0
    return np.array([P, Gs, P + Gs, rho, V, du], dtype=np.float64)
