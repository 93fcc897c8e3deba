"""Fourier-domain preconditioners (thesis §4.3, §4.3.1, §4.4).

* Periodic Laplacian (§4.3): M_2 u = u * kappa_Delta (periodic convolution with
  the 5-point kernel), whose 2-D DFT symbol is
  lambda_Delta(k1, k2) = 4 sin^2(pi k1 / n) + 4 sin^2(pi k2 / n).
  (The printed symbol repeats the first index; the derivation just above it
  gives one term per axis, which is the reading taken.)
* Inverse-norm preconditioner (§4.3.1): tilde M = F^{-1} (1/||x||_eps) F with
  ||x||_eps = sqrt(||x||^2 + eps^2).  Reading of "x": the centred integer DFT
  frequency (f(k1), f(k2)), f(k) = k for k <= n/2 and k - n otherwise.
* The PDRQS1 multiplier (§4.4):
  M^{-1} y = F^{-1}( F(y) * rho / (sigma^2 c + (sigma tau)^2 lambda_Delta rho) )
  with rho = ||x||_eps.  Reading: the algorithm prints ||x|| without eps, which
  would zero the multiplier at the zero frequency so that the image mean never
  updates; §4.3.1 defines the eps-regularized norm for exactly this purpose,
  and the unconstrained variant PDRQS2 uses it, so rho = ||x||_eps here.
"""
from __future__ import annotations

import numpy as np


def freq_index(n: int) -> np.ndarray:
    """Centred integer DFT frequency of bin k: k for k <= n/2, else k - n."""
    k = np.arange(n)
    return np.where(k <= n // 2, k, k - n).astype(np.float64)


def rho_eps(n: int, eps: float) -> np.ndarray:
    """||x||_eps = sqrt(f(k1)^2 + f(k2)^2 + eps^2) on the (n, n) DFT grid."""
    f = freq_index(n)
    return np.sqrt(f[:, None] ** 2 + f[None, :] ** 2 + eps * eps)


def lap_symbol(n: int) -> np.ndarray:
    """lambda_Delta(k1, k2) = 4 sin^2(pi k1/n) + 4 sin^2(pi k2/n)  (§4.3)."""
    s = 4.0 * np.sin(np.pi * np.arange(n) / n) ** 2
    return s[:, None] + s[None, :]


def multiplier(n: int, sigma: float, tau: float, c: float, eps: float) -> np.ndarray:
    """rho / (sigma^2 c + (sigma tau)^2 lambda_Delta rho)  (§4.4, PDRQS1)."""
    r = rho_eps(n, eps)
    return r / (sigma * sigma * c + (sigma * tau) ** 2 * lap_symbol(n) * r)


def apply_multiplier(y: np.ndarray, mult: np.ndarray) -> np.ndarray:
    """F^{-1}(mult * F(y)), real part (mult is real and even, so the result is real)."""
    return np.real(np.fft.ifft2(mult * np.fft.fft2(np.asarray(y, dtype=np.float64))))


def precond_inverse(y: np.ndarray, sigma: float, tau: float, c: float, eps: float) -> np.ndarray:
    """x = M^{-1} y for the PDRQS1 preconditioner  (§4.4)."""
    return apply_multiplier(y, multiplier(y.shape[0], sigma, tau, c, eps))


def sqrt_inv_norm_precond(y: np.ndarray, eps: float) -> np.ndarray:
    """tilde M^{-1/2} y = F^{-1}( sqrt(rho) F(y) ): the symmetric square root of
    the inverse of tilde M = F^{-1}(1/rho)F  (§4.3.1)."""
    return apply_multiplier(y, np.sqrt(rho_eps(y.shape[0], eps)))


# ---------------------------------------------------------------------------
# Variants (thesis §4.3 Richardson, §4.5 non-negativity).

def multiplier_nonneg(n: int, sigma: float, tau: float, c: float, eps: float) -> np.ndarray:
    """rho / (rho + sigma^2 c + (sigma tau)^2 lambda_Delta rho)  (§4.5): the
    inverse of M = id + c sigma^2 tilde M - (sigma tau)^2 Delta_p."""
    r = rho_eps(n, eps)
    return r / (r + sigma * sigma * c + (sigma * tau) ** 2 * lap_symbol(n) * r)
