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


# ---------------------------------------------------------------------------
# Circulant preconditioner (§4.3.3, after Ramani-Fessler).
#
# A^* A is approximated by a circulant matrix on the vectorized image: the
# image is flattened to a length-L vector (L = n^2), the response of A^* A to
# the impulse at the centre pixel is taken as the circulant's first column,
# and M^{-1} u = F_L^{-1}(F_L(u) / F_L(K)) with the 1-D DFT F_L.  Readings:
#  * vectorization: column-major, index m = j + n i for pixel (row j, column i)
#    (the column-stacking order of the thesis' MATLAB code);
#  * the impulse at pixel (n/2, n/2), m0 = n/2 + n (n/2); the circulant's
#    column is the response shifted to index 0, c_m = k~_{(m + m0) mod L},
#    symmetrized as printed, k_m = (c_m + c_{(L - m) mod L}) / 2;
#  * the Laplace kernel from -Delta_h applied to the same impulse: 4 at
#    index 0 and -1 at +-1 (rows) and +-n (columns), symbol
#    4 - 2 cos(2 pi q / L) - 2 cos(2 pi q / n);
#  * K = alpha k + beta kappa_Delta (alpha = sigma^2, beta = (sigma tau)^2)
#    and, as for the impulse-response preconditioner, M = c M_K with
#    c = c_safety lambda_max(M_K^{-1} T).

def flatten(u: np.ndarray) -> np.ndarray:
    """Column-major vector of an (n, n) image stored u[j, i]: m = j + n i."""
    return np.asarray(u, dtype=np.float64).ravel(order="F")


def unflatten(x: np.ndarray, n: int) -> np.ndarray:
    return np.asarray(x).reshape((n, n), order="F")


def circulant_kernel(A, At, n: int) -> np.ndarray:
    """Symmetrized, origin-shifted column of the circulant approximation of A^* A."""
    L = n * n
    d = np.zeros((n, n))
    d[n // 2, n // 2] = 1.0
    kt = flatten(At(A(d)))
    m0 = n // 2 + n * (n // 2)
    c = np.roll(kt, -m0)
    return 0.5 * (c + c[(L - np.arange(L)) % L])


def circulant_lap_symbol(n: int) -> np.ndarray:
    L = n * n
    q = np.arange(L)
    return 4.0 - 2.0 * np.cos(2 * np.pi * q / L) - 2.0 * np.cos(2 * np.pi * q / n)


def circulant_full_symbol(k: np.ndarray, alpha: float, beta: float) -> np.ndarray:
    """F_L(K) = alpha F_L(k) + beta F_L(kappa_Delta) (real: k is symmetric)."""
    n = int(round(np.sqrt(k.size)))
    return alpha * np.real(np.fft.fft(k)) + beta * circulant_lap_symbol(n)


def apply_circulant(u: np.ndarray, symbol_inv: np.ndarray) -> np.ndarray:
    """F_L^{-1}(symbol_inv * F_L(u)) on the vectorized image, back as an image."""
    n = u.shape[0]
    x = np.fft.ifft(symbol_inv * np.fft.fft(flatten(u)))
    return unflatten(np.real(x), n)
