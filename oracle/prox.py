"""Pointwise resolvents (thesis §3.3, §4.4; variants §3.5, §4.5).

Sinogram part of G^* (§3.3 lemmas on g*_{1,1}, g*_{1,2} and their resolvents;
the same closed forms with step sigma in §4.4):
  off the metal trace D0:  (q - s u0) / (1 + s)       (L2 fit)
  on D0:                   min(q - s C, 0)            (inequality R u >= C)
with step s (tau in Algorithm CP, sigma in PDRQS1).  C may vary per bin
(§3.5, location-dependent threshold).

TV part: projection onto the pointwise Euclidean ball of the given radius,
w / max(1, |w| / radius).  In Algorithm CP the radius is lambda; in PDRQS1
the operator is K_2 = tau nabla_h, so G_2 = (lambda/tau)||.||_1 and the radius
is lambda/tau, which is what the algorithm's max(1, tau |.| / lambda) means.
"""
from __future__ import annotations

import numpy as np


def prox_sino(q: np.ndarray, step: float, u0: np.ndarray, bound: np.ndarray,
              mask: np.ndarray) -> np.ndarray:
    """Resolvent (id + step dG_1^*)^{-1}(q), pointwise (§3.3 / §4.4)."""
    fit = (q - step * u0) / (1.0 + step)
    clamp = np.minimum(q - step * bound, 0.0)
    return np.where(mask, clamp, fit)


def tv_project(q: np.ndarray, radius: float) -> np.ndarray:
    """Pointwise projection of the 2-vector field q (shape (2, n, n)) onto the
    ball of the given radius: q / max(1, |q| / radius)  (§3.3)."""
    nrm = np.sqrt(q[0] ** 2 + q[1] ** 2)
    # q / max(1, |q|/radius), written so that radius = 0 (lambda = 0) projects onto {0}
    scale = np.where(nrm > radius, radius / np.where(nrm > 0, nrm, 1.0), 1.0)
    return q * scale


# ---------------------------------------------------------------------------
# Variants (§3.5, §4.5).

def prox_sino_weighted(q, step, u0, weight, bound, mask):
    """Weighted fit (1/2) w (x - u0)^2 off D0 (§3.5, weighted fitting):
    resolvent of its conjugate (1/(2w)) xi^2 + xi u0 is (q - step u0)/(1 + step/w)."""
    fit = (q - step * u0) / (1.0 + step / weight)
    return np.where(mask, np.minimum(q - step * bound, 0.0), fit)


def prox_sino_ignore(q, step, u0, mask):
    """Ignoring data on D0 (§3.5): G_1 has no term there, its conjugate is the
    indicator of {0}, whose resolvent is 0."""
    return np.where(mask, 0.0, (q - step * u0) / (1.0 + step))


def prox_sino_fit_everywhere(q, step, u0, bound, mask):
    """Fit everywhere plus the constraint on D0 (§3.5): on D0 the function
    (1/2)(x - u0)^2 + I{x >= C}.  Its resolvent of the conjugate, by the Moreau
    identity, is q - step * prox_{g/step}(q/step), where prox_{g/step}(z) is
    the clipped quadratic minimizer max((step z + u0)/(step + 1), C)."""
    z = q / step
    primal = np.maximum((step * z + u0) / (step + 1.0), bound)
    on_d0 = q - step * primal
    return np.where(mask, on_d0, (q - step * u0) / (1.0 + step))


def prox_sino_hard(q, step, u0, bound, mask):
    """Hard constraint R u = u0 off D0 (§3.5): conjugate of I{x = u0} is
    xi u0, whose resolvent is q - step u0; the inequality on D0 as before."""
    return np.where(mask, np.minimum(q - step * bound, 0.0), q - step * u0)


def prox_nonneg(y: np.ndarray, d: float = 0.0) -> np.ndarray:
    """Resolvent of the indicator of [d, inf): max(y, d)  (§4.5)."""
    return np.maximum(y, d)
