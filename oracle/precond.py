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


# ---------------------------------------------------------------------------
# Impulse-response preconditioner (§4.3.2).
#
# The response of A^* A to a unit impulse at pixel (n/2, n/2) (n even) is
# taken as a convolution kernel: k~ = A^* A delta.  Readings:
#  * the kernel of a periodic deconvolution has its centre at the origin, so
#    k~ is read centred on the impulse: k(x) = k~(n/2 + x) with x taken
#    modulo n (the thesis leaves the shift implicit);
#  * "k = 1/2 (k~ + k~^T) to guarantee a symmetric preconditioner": the
#    average over the eight symmetries of the square about the origin
#    (transposition as printed, and the two axis mirrors).  It contains the
#    printed average, makes k point symmetric (so that deconvolution by it is
#    a symmetric operator, F(k) real) and even in each axis, as the other
#    multipliers are;
#  * with T = alpha A^* A - beta Delta_h (alpha = sigma^2, beta = (sigma tau)^2
#    for PDRQS1) the full kernel K = alpha k + beta kappa_Delta has the real
#    symbol F(K) = alpha F(k) + beta lambda_Delta, and the preconditioner is
#    c M_K with M_K = F^{-1} F(K) F, c = c_safety lambda_max(M_K^{-1} T) (the
#    constant of "c M - T >= 0" scales the whole M here, as printed).
#  F(k) itself can dip below zero at the highest frequencies (the
#  interpolation's response); F(K) must be positive, which the setup checks.

def center_and_symmetrize(kt: np.ndarray) -> np.ndarray:
    """k(x) = mean over the 8 symmetries g of the square of k~(n/2 + g x),
    indices modulo n."""
    n = kt.shape[0]
    kc = np.roll(kt, (-(n // 2), -(n // 2)), axis=(0, 1))   # k~(n/2 + x) at x
    out = np.zeros_like(kc, dtype=np.float64)
    idx = np.arange(n)
    neg = (-idx) % n
    for base in (kc, kc.T):
        for ry in (idx, neg):
            for rx in (idx, neg):
                out += base[np.ix_(ry, rx)]
    return out / 8.0


def impulse_kernel(A, At, n: int) -> np.ndarray:
    """The symmetrized, origin-centred response k of A^* A to delta at (n/2, n/2)."""
    d = np.zeros((n, n))
    d[n // 2, n // 2] = 1.0
    return center_and_symmetrize(At(A(d)))


def kernel_symbol(k: np.ndarray) -> np.ndarray:
    """F(k) for a real kernel that is even in each axis (real-valued)."""
    f = np.fft.fft2(k)
    return np.real(f)


def impulse_full_symbol(khat: np.ndarray, alpha: float, beta: float) -> np.ndarray:
    """F(K) = alpha F(k) + beta lambda_Delta."""
    return alpha * khat + beta * lap_symbol(khat.shape[0])


def impulse_multiplier(fK: np.ndarray, c: float) -> np.ndarray:
    """(c M_K)^{-1} as a Fourier multiplier: 1 / (c F(K))."""
    return 1.0 / (c * fK)
