"""Pins of the oracle's gradient/divergence/TV (thesis §3.1), preconditioner
(§4.3, §4.3.1, §4.4) and resolvents (§3.3, §3.5, §4.5)."""
import math

import numpy as np
import pytest
from scipy import optimize

from oracle import geometry, power, precond, prox, radon, tv


def _grad_matrix(n):
    cols = []
    for k in range(n * n):
        e = np.zeros(n * n)
        e[k] = 1.0
        cols.append(tv.grad(e.reshape(n, n)).ravel())
    return np.array(cols).T


def test_grad_div_adjoint():
    """<nabla_h u, p> = <u, -div_h p> (§3.1)."""
    rng = np.random.default_rng(0)
    for n, h in ((7, 1.0), (16, 0.5)):
        u = rng.standard_normal((n, n))
        p = rng.standard_normal((2, n, n))
        lhs = np.sum(tv.grad(u, h) * p)
        rhs = -np.sum(u * tv.div(p, h))
        assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(lhs))


def test_grad_norm_closed_form():
    """||nabla_h||^2 = (8/h^2) cos^2(pi/(2n)) < 8/h^2 (§3.1 bound; the closed
    form follows from the Neumann Laplacian being diagonalized by the DCT-II),
    and nabla_h u = 0 exactly for constants."""
    for n in (4, 6, 9):
        G = _grad_matrix(n)
        smax2 = np.linalg.eigvalsh(G.T @ G)[-1]
        assert smax2 == pytest.approx(8 * math.cos(math.pi / (2 * n)) ** 2, rel=1e-12)
        # null space = constants
        ev = np.linalg.eigvalsh(G.T @ G)
        assert abs(ev[0]) < 1e-12 and ev[1] > 1e-6
    assert np.all(tv.grad(np.full((5, 5), 3.7)) == 0.0)


def test_tv_of_rectangle():
    """TV of an a-wide, b-tall block of height d away from the border is
    |d| (2a + 2b - 2 + sqrt(2)) with forward differences (§3.1): the column
    left of the block and the block's last column carry an x-jump (2b - 1
    pixels with a single jump), the row above and the block's last row a
    y-jump (2a - 1 pixels), and the block's far corner pixel carries both
    (|d| sqrt(2)).  TV of a constant is zero."""
    n, a, b, d = 20, 5, 7, 2.5
    u = np.zeros((n, n))
    u[4:4 + b, 6:6 + a] = d
    expect = abs(d) * (2 * a + 2 * b - 2 + math.sqrt(2))
    assert tv.tv(u) == pytest.approx(expect, rel=1e-14)
    assert tv.tv(np.full((n, n), -1.3)) == 0.0


def test_periodic_laplacian_symbol():
    """The DFT of the periodic 5-point kernel is 4 sin^2(pi k1/n) + 4 sin^2(pi k2/n) (§4.3)."""
    for n in (6, 8, 12):
        k = np.zeros((n, n))
        k[0, 0] = 4
        k[0, 1] = k[1, 0] = k[0, -1] = k[-1, 0] = -1
        f = np.fft.fft2(k)
        assert np.max(np.abs(f.imag)) < 1e-12
        assert np.allclose(f.real, precond.lap_symbol(n), atol=1e-12)


def test_periodic_laplacian_dominates_neumann():
    """<(-Delta_p + Delta_h) u, u> >= 0 (§4.3): the periodic Laplacian is a
    valid preconditioner term for -Delta_h = nabla_h^* nabla_h."""
    n = 6
    G = _grad_matrix(n)
    neg_lap_h = G.T @ G
    lp = np.zeros((n * n, n * n))
    for k in range(n * n):
        e = np.zeros(n * n)
        e[k] = 1.0
        lp[:, k] = precond.apply_multiplier(e.reshape(n, n), precond.lap_symbol(n)).ravel()
    # independent construction of -Delta_p by np.roll stencils
    def neg_lap_p(u):
        return 4 * u - np.roll(u, 1, 0) - np.roll(u, -1, 0) - np.roll(u, 1, 1) - np.roll(u, -1, 1)
    for k in range(n * n):
        e = np.zeros(n * n)
        e[k] = 1.0
        assert np.allclose(lp[:, k], neg_lap_p(e.reshape(n, n)).ravel(), atol=1e-12)
    assert np.linalg.eigvalsh(lp - neg_lap_h)[0] > -1e-10


def test_multiplier_properties():
    """The PDRQS1 multiplier is real, positive, even in each frequency and its
    operator is symmetric positive definite (needed for M^{-1} to map real
    images to real images and for the convergence theory of §4.1)."""
    n = 12
    m = precond.multiplier(n, 1.0, 0.35, 2.0, 0.3)
    assert np.all(m > 0)
    f = precond.freq_index(n)
    assert np.all(np.abs(f) <= n / 2)
    # evenness: m(k1, k2) = m(-k1, k2) = m(k1, -k2)
    idx = (-np.arange(n)) % n
    assert np.allclose(m, m[idx, :]) and np.allclose(m, m[:, idx])
    y = np.random.default_rng(1).standard_normal((n, n))
    x = precond.apply_multiplier(y, m)
    assert np.max(np.abs(np.imag(np.fft.ifft2(m * np.fft.fft2(y))))) < 1e-12
    assert np.sum(x * y) > 0


def test_preconditioner_inverts_its_operator():
    """M^{-1} of §4.4 inverts M = sigma^2 c tilde M + (sigma tau)^2 (-Delta_p),
    with tilde M applied as F^{-1}(F(.)/rho_eps) and -Delta_p by stencil."""
    n, sigma, tau, c, eps = 10, 0.8, 0.4, 3.0, 0.3
    rng = np.random.default_rng(2)
    u = rng.standard_normal((n, n))
    tm = precond.apply_multiplier(u, 1.0 / precond.rho_eps(n, eps))
    lp = 4 * u - np.roll(u, 1, 0) - np.roll(u, -1, 0) - np.roll(u, 1, 1) - np.roll(u, -1, 1)
    Mu = sigma ** 2 * c * tm + (sigma * tau) ** 2 * lp
    assert np.allclose(precond.precond_inverse(Mu, sigma, tau, c, eps), u, atol=1e-11)


def test_preconditioner_feasible_after_c_selection():
    """With c = 1.1 lambda_max(tilde M^{-1} A^* A) from power iteration,
    M - sigma^2 K^* K >= 0 (the PDRQ condition for the pure linear-quadratic
    case, §4.1.1 / §4.4), checked by dense eigendecomposition."""
    g = geometry.Geometry(8, 10, 14)
    A = radon.radon_matrix(g)
    beta = np.linalg.svd(A, compute_uv=False)[0]
    A = A / beta
    n = g.n
    G = _grad_matrix(n)
    sigma, tau, eps = 1.0, 1 / math.sqrt(8), 0.3
    rng = np.random.default_rng(3)
    lmax = power.precond_constant_eig(lambda u: (A @ u.ravel()).reshape(g.n_angles, g.n_bins),
                                      lambda v: (A.T @ v.ravel()).reshape(n, n),
                                      rng.standard_normal((n, n)), eps, iters=200)
    c = 1.1 * lmax
    Minv = np.zeros((n * n, n * n))
    for k in range(n * n):
        e = np.zeros(n * n)
        e[k] = 1.0
        Minv[:, k] = precond.precond_inverse(e.reshape(n, n), sigma, tau, c, eps).ravel()
    Mmat = np.linalg.inv(Minv)
    T = sigma ** 2 * (A.T @ A + tau ** 2 * G.T @ G)
    assert np.linalg.eigvalsh(0.5 * (Mmat + Mmat.T) - T)[0] > -1e-9
    # and the estimate matches the dense eigenvalue of tilde M^{-1} A^* A
    S = np.zeros((n * n, n * n))
    for k in range(n * n):
        e = np.zeros(n * n)
        e[k] = 1.0
        S[:, k] = precond.sqrt_inv_norm_precond(e.reshape(n, n), eps).ravel()
    dense = np.linalg.eigvalsh(S @ A.T @ A @ S)[-1]
    assert lmax == pytest.approx(dense, rel=1e-6)


# ---------------------------------------------------------------------------
# resolvents: closed forms against numerical minimization of
# 1/2 (x - v)^2 + s g^*(x), with g^* written out from the definition of the
# convex conjugate as a supremum evaluated numerically.

def _conj_numeric(g, xi, lo=-60, hi=60):
    res = optimize.minimize_scalar(lambda z: -(xi * z - g(z)), bounds=(lo, hi), method="bounded",
                                   options={"xatol": 1e-11})
    return -res.fun


def test_prox_l2_fit_numeric():
    u0, s = 0.7, 0.9
    g = lambda z: 0.5 * (z - u0) ** 2
    for v in (-2.0, 0.3, 1.8):
        obj = lambda x: 0.5 * (x - v) ** 2 + s * _conj_numeric(g, x)
        xnum = optimize.minimize_scalar(obj, bounds=(-10, 10), method="bounded",
                                        options={"xatol": 1e-10}).x
        got = prox.prox_sino(np.array(v), s, np.array(u0), np.array(0.0), np.array(False))
        assert float(got) == pytest.approx(xnum, abs=1e-6)


def test_prox_inequality_numeric():
    """Resolvent of the conjugate of I{z >= C}: min(v - s C, 0) (§3.3)."""
    C, s = 1.3, 0.8
    for v in (-1.0, 0.5, 1.0, 3.0):
        # g^*(xi) = xi C for xi <= 0, +inf otherwise (evaluated by its definition)
        def conj(xi):
            return xi * C if xi <= 0 else np.inf
        obj = lambda x: 0.5 * (x - v) ** 2 + s * (x * C if x <= 0 else 1e9 * x)
        xnum = optimize.minimize_scalar(obj, bounds=(-10, 10), method="bounded",
                                        options={"xatol": 1e-10}).x
        got = prox.prox_sino(np.array(v), s, np.array(0.0), np.array(C), np.array(True))
        assert float(got) == pytest.approx(xnum, abs=1e-6)
        assert conj(float(got)) < np.inf


def test_moreau_identity():
    """prox_{s g^*}(v) + s prox_{g/s}(v/s) = v (§1.3 Moreau identity), with
    prox_{g/s} written as the plain minimizer of the primal function."""
    rng = np.random.default_rng(4)
    v = rng.standard_normal(50) * 3
    u0 = rng.standard_normal(50)
    C = rng.uniform(0, 1, 50)
    for s in (0.3, 1.0, 2.5):
        # primal prox of 1/2 (z - u0)^2 with weight 1/s: (s x + u0) / (s + 1)
        p_fit = (s * (v / s) + u0) / (s + 1.0)
        # primal prox of I{z >= C}: projection max(x, C)
        p_ineq = np.maximum(v / s, C)
        got_fit = prox.prox_sino(v, s, u0, C, np.zeros(50, bool))
        got_ineq = prox.prox_sino(v, s, u0, C, np.ones(50, bool))
        assert np.allclose(got_fit + s * p_fit, v, atol=1e-13)
        assert np.allclose(got_ineq + s * p_ineq, v, atol=1e-13)


def test_tv_projection_numeric():
    """Pointwise projection onto the Euclidean ball of radius r: compared with
    a brute-force search on a fine polar grid."""
    rng = np.random.default_rng(5)
    q = rng.standard_normal((2, 3, 3)) * 2
    r = 1.1
    got = prox.tv_project(q, r)
    rad = np.linspace(0, r, 2001)
    ang = np.linspace(0, 2 * np.pi, 4001)
    R, T = np.meshgrid(rad, ang)
    px, py = R * np.cos(T), R * np.sin(T)
    for j in range(3):
        for i in range(3):
            d = (px - q[0, j, i]) ** 2 + (py - q[1, j, i]) ** 2
            k = np.unravel_index(np.argmin(d), d.shape)
            assert got[0, j, i] == pytest.approx(px[k], abs=2e-3)
            assert got[1, j, i] == pytest.approx(py[k], abs=2e-3)
            assert np.hypot(got[0, j, i], got[1, j, i]) <= r + 1e-12


def test_prox_variants_numeric():
    """Weighted fit, ignoring data, fit everywhere with the constraint, hard
    constraint (§3.5) and non-negativity (§4.5), each against numerical
    minimization with the conjugate evaluated from its definition."""
    u0, C, wgt = 0.6, 1.1, 2.5
    for s in (0.5, 1.7):
        for v in (-2.5, -0.4, 0.9, 2.2, 4.0):
            def solve(gfun, lo=-20, hi=20):
                obj = lambda x: 0.5 * (x - v) ** 2 + s * _conj_numeric(gfun, x)
                return optimize.minimize_scalar(obj, bounds=(lo, hi), method="bounded",
                                                options={"xatol": 1e-9}).x
            a = np.array
            got = prox.prox_sino_weighted(a(v), s, a(u0), a(wgt), a(C), a(False))
            assert float(got) == pytest.approx(solve(lambda z: 0.5 * wgt * (z - u0) ** 2), abs=1e-5)
            # fit everywhere on D0: f(z) = 1/2 (z - u0)^2 + I{z >= C}
            f_fe = lambda z: 0.5 * (z - u0) ** 2 + (0.0 if z >= C else 1e6 * (C - z) ** 2 + 1e3 * (C - z))
            got = prox.prox_sino_fit_everywhere(a(v), s, a(u0), a(C), a(True))
            assert float(got) == pytest.approx(solve(f_fe), abs=1e-3)
    got = prox.prox_sino_ignore(np.array([1.0, 2.0]), 0.5, np.array([0.3, 0.3]), np.array([True, False]))
    assert got[0] == 0.0 and got[1] == pytest.approx((2.0 - 0.15) / 1.5)
    got = prox.prox_sino_hard(np.array([1.0]), 0.5, np.array([0.3]), np.array([0.0]), np.array([False]))
    assert got[0] == pytest.approx(1.0 - 0.15)
    assert np.array_equal(prox.prox_nonneg(np.array([-1.0, 0.0, 2.0])), [0.0, 0.0, 2.0])
