"""Power iterations (thesis §4.3, §4.3.1, §5.1).

The thesis obtains these operator constants with power iterations but does
not fix the step count; the reading here is 30 steps, a stated start vector (drawn by the
caller from the seeded input generator and passed in), and the estimate
||B x_{29}|| with x_{29} the unit-norm iterate before the last application.

* ||R_h||^2 = lambda_max(R_h^* R_h)  (the normalization of §5.1, in place of
  the crude bound of the lemma on ||R_h|| in §3.1).
* lambda_max(tilde M^{-1} A^* A) = lambda_max(tilde M^{-1/2} A^* A tilde M^{-1/2})
  for the inverse-norm preconditioner (§4.3.1: c is chosen larger than the
  largest eigenvalue of tilde M^{-1} R_h^* R_h, here of the normalized A).
"""
from __future__ import annotations

from typing import Callable

import numpy as np

from . import precond


def power_max_eig(op: Callable[[np.ndarray], np.ndarray], x0: np.ndarray,
                  iters: int = 30) -> float:
    """Largest eigenvalue of a symmetric positive semi-definite operator.

    x <- op(x) / ||op(x)|| for `iters` steps starting from x0 / ||x0||; the
    estimate is ||op(x)|| at the last step (x of unit norm).
    """
    x = np.asarray(x0, dtype=np.float64)
    x = x / np.linalg.norm(x)
    lam = 0.0
    for _ in range(iters):
        y = op(x)
        lam = float(np.linalg.norm(y))
        x = y / lam
    return lam


def radon_norm(fwd, adj, x0: np.ndarray, iters: int = 30) -> float:
    """beta_R = sqrt(lambda_max(R_h^* R_h)) by power iteration."""
    return float(np.sqrt(power_max_eig(lambda x: adj(fwd(x)), x0, iters)))


def precond_constant_eig(fwd_a, adj_a, x0: np.ndarray, eps: float, iters: int = 30) -> float:
    """lambda_max(tilde M^{-1/2} A^* A tilde M^{-1/2}) by power iteration (§4.3.1)."""
    def op(x):
        z = precond.sqrt_inv_norm_precond(x, eps)
        z = adj_a(fwd_a(z))
        return precond.sqrt_inv_norm_precond(z, eps)
    return power_max_eig(op, x0, iters)


def impulse_constant_eig(fwd_a, adj_a, fK: np.ndarray, alpha: float, beta: float, h: float,
                         x0: np.ndarray, iters: int = 30) -> float:
    """lambda_max(M_K^{-1} T) = lambda_max(M_K^{-1/2} T M_K^{-1/2}) for the
    impulse-response preconditioner (§4.3.2), T = alpha A^* A - beta div nabla."""
    from . import tv
    s = 1.0 / np.sqrt(fK)

    def op(x):
        y = precond.apply_multiplier(x, s)
        t = alpha * adj_a(fwd_a(y)) - beta * tv.div(tv.grad(y, h), h)
        return precond.apply_multiplier(t, s)

    return power_max_eig(op, x0, iters)


def circulant_constant_eig(fwd_a, adj_a, fK: np.ndarray, alpha: float, beta: float, h: float,
                           x0: np.ndarray, iters: int = 30) -> float:
    """lambda_max(M_K^{-1} T) for the circulant preconditioner (§4.3.3)."""
    from . import tv
    s = 1.0 / np.sqrt(fK)

    def op(x):
        y = precond.apply_circulant(x, s)
        t = alpha * adj_a(fwd_a(y)) - beta * tv.div(tv.grad(y, h), h)
        return precond.apply_circulant(t, s)

    return power_max_eig(op, x0, iters)
