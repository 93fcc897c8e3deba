"""Pins of the impulse-response preconditioner (§4.3.2, no GPU): for an
operator that is a periodic convolution the impulse kernel's symbol is the
exact one, the symmetrization is the D4 average, c M_K dominates T (dense
check), and PDRQS1 with it reaches Algorithm CP's minimizer."""
import numpy as np
import pytest

from oracle import cp, geometry, pdrq, power, precond, radon, tv


def _d4_kernel(n, seed):
    rng = np.random.default_rng(seed)
    h = np.zeros((n, n))
    h[:3, :3] = rng.uniform(0.2, 1.0, (3, 3))
    return precond.center_and_symmetrize(np.roll(h, (n // 2, n // 2), axis=(0, 1)))


def test_impulse_kernel_of_a_convolution_is_exact():
    # A u = h (*) u (periodic), h symmetric under the square's symmetries:
    # A^* A is the convolution with h (*) h, whose symbol is F(h)^2
    n = 16
    h = _d4_kernel(n, 0)
    H = np.fft.fft2(h)
    A = lambda u: np.real(np.fft.ifft2(H * np.fft.fft2(u)))
    At = lambda v: np.real(np.fft.ifft2(np.conj(H) * np.fft.fft2(v)))
    k = precond.impulse_kernel(A, At, n)
    assert np.allclose(precond.kernel_symbol(k), np.abs(H) ** 2, atol=1e-12)


def test_symmetrization_is_the_d4_average():
    n = 12
    kt = np.random.default_rng(1).standard_normal((n, n))
    k = precond.center_and_symmetrize(kt)
    neg = (-np.arange(n)) % n
    assert np.allclose(k, k.T)
    assert np.allclose(k, k[neg, :])
    assert np.allclose(k, k[:, neg])
    # idempotent once re-centred at the impulse, and F(k) is real
    again = precond.center_and_symmetrize(np.roll(k, (n // 2, n // 2), axis=(0, 1)))
    assert np.allclose(again, k)
    assert np.max(np.abs(np.fft.fft2(k).imag)) < 1e-12


@pytest.fixture(scope="module")
def tiny():
    g = geometry.Geometry(8, 12, 16)
    R = radon.radon_matrix(g)
    fwd = lambda u: (R @ u.ravel()).reshape(g.n_angles, g.n_bins)
    adj = lambda v: (R.T @ v.ravel()).reshape(g.n, g.n)
    rng = np.random.default_rng(2)
    ut = np.zeros((8, 8))
    ut[2:6, 2:7] = 1.0
    u0 = fwd(ut) + 0.05 * rng.standard_normal((12, 16))
    mask = np.zeros((12, 16), dtype=bool)
    prob = pdrq.Problem(g, u0, mask, np.zeros((12, 16)), lam=0.5)
    s = pdrq.setup(prob, pdrq.Params(), rng.standard_normal((8, 8)), rng.standard_normal((8, 8)),
                   fwd=fwd, adj=adj, kind="impulse")
    return s, R


def test_c_makes_the_preconditioner_dominate_T(tiny):
    s, R = tiny
    n = s.problem.geom.n
    sig, tau = s.params.sigma, s.params.tau
    A = R / s.beta
    G = np.array([tv.grad(np.eye(n * n)[k].reshape(n, n), 1.0).ravel() for k in range(n * n)]).T
    T = sig * sig * A.T @ A + (sig * tau) ** 2 * G.T @ G
    # M = (multiplier)^{-1} as a dense matrix from its action on unit images
    Minv = np.array([precond.apply_multiplier(np.eye(n * n)[k].reshape(n, n), s.mult).ravel()
                     for k in range(n * n)]).T
    M = np.linalg.inv(Minv)
    assert np.allclose(M, M.T, atol=1e-10)
    assert np.linalg.eigvalsh(0.5 * (M + M.T) - T).min() >= -1e-10


def test_pdrqs1_with_impulse_preconditioner_reaches_cp_minimizer(tiny):
    s, _ = tiny
    mask = s.problem.mask
    u_cp, _, _ = cp.run(s.A, s.At, s.b, s.cb, mask, s.lam_t, 8, 20000, 0.32, 0.32)
    st = pdrq.zero_state(s)
    for _ in range(3000):
        st = pdrq.step(s, st)
    assert np.max(np.abs(st.u - u_cp)) < 1e-8


def test_full_symbol_positive_on_a_realistic_geometry():
    g = geometry.Geometry(32, 45, 48)
    fwd = lambda u: radon.radon_fwd(g, u)
    adj = lambda v: radon.radon_adj(g, v)
    beta = power.radon_norm(fwd, adj, np.random.default_rng(3).standard_normal((32, 32)), 40)
    khat = precond.kernel_symbol(precond.impulse_kernel(lambda u: fwd(u) / beta,
                                                        lambda v: adj(v) / beta, 32))
    fK = precond.impulse_full_symbol(khat, 1.0, 1.0 / 8.0)
    assert fK.min() > 0
    # the impulse response of the normalized A^* A has a symbol near 1 at low frequencies
    assert 0.2 < khat[0, 0] < 20


# --- circulant preconditioner (§4.3.3) --------------------------------------

def test_circulant_kernel_of_a_circulant_operator_is_exact():
    # A = a circulant on the column-major vectorized image with a symmetric
    # first column h: A^* A is the circulant of h (*) h, symbol |F_L(h)|^2
    n = 8
    L = n * n
    rng = np.random.default_rng(4)
    h = np.zeros(L)
    h[:5] = rng.uniform(0.2, 1.0, 5)
    h = 0.5 * (h + h[(L - np.arange(L)) % L])
    Hs = np.fft.fft(h)
    A = lambda u: precond.unflatten(np.real(np.fft.ifft(Hs * np.fft.fft(precond.flatten(u)))), n)
    At = lambda v: precond.unflatten(np.real(np.fft.ifft(np.conj(Hs) * np.fft.fft(precond.flatten(v)))), n)
    k = precond.circulant_kernel(A, At, n)
    assert np.allclose(np.fft.fft(k).real, np.abs(Hs) ** 2, atol=1e-12)
    # the Laplace kernel's symbol: the 1-D DFT of 4, -1 at +-1 and +-n
    kap = np.zeros(L)
    kap[0] = 4.0
    kap[[1, L - 1, n, L - n]] = -1.0
    assert np.allclose(np.fft.fft(kap).real, precond.circulant_lap_symbol(n), atol=1e-12)


def test_vectorization_is_column_major():
    u = np.arange(6.0).reshape(2, 3)   # u[j, i]: index j + 2 i
    assert list(precond.flatten(u)) == [0.0, 3.0, 1.0, 4.0, 2.0, 5.0]
    sq = np.arange(9.0).reshape(3, 3)
    assert np.array_equal(precond.unflatten(precond.flatten(sq), 3), sq)


@pytest.fixture(scope="module")
def tiny_circ():
    g = geometry.Geometry(8, 12, 16)
    R = radon.radon_matrix(g)
    fwd = lambda u: (R @ u.ravel()).reshape(g.n_angles, g.n_bins)
    adj = lambda v: (R.T @ v.ravel()).reshape(g.n, g.n)
    rng = np.random.default_rng(2)
    ut = np.zeros((8, 8))
    ut[2:6, 2:7] = 1.0
    u0 = fwd(ut) + 0.05 * rng.standard_normal((12, 16))
    mask = np.zeros((12, 16), dtype=bool)
    prob = pdrq.Problem(g, u0, mask, np.zeros((12, 16)), lam=0.5)
    s = pdrq.setup(prob, pdrq.Params(), rng.standard_normal((8, 8)), rng.standard_normal((8, 8)),
                   fwd=fwd, adj=adj, kind="circulant")
    return s, R


def test_circulant_c_makes_the_preconditioner_dominate_T(tiny_circ):
    s, R = tiny_circ
    n = s.problem.geom.n
    sig, tau = s.params.sigma, s.params.tau
    A = R / s.beta
    G = np.array([tv.grad(np.eye(n * n)[k].reshape(n, n), 1.0).ravel() for k in range(n * n)]).T
    T = sig * sig * A.T @ A + (sig * tau) ** 2 * G.T @ G
    Minv = np.array([pdrq.apply_precond(s, np.eye(n * n)[k].reshape(n, n)).ravel()
                     for k in range(n * n)]).T
    M = np.linalg.inv(Minv)
    assert np.allclose(M, M.T, atol=1e-10)
    assert np.linalg.eigvalsh(0.5 * (M + M.T) - T).min() >= -1e-10


def test_pdrqs1_with_circulant_preconditioner_reaches_cp_minimizer(tiny_circ):
    s, _ = tiny_circ
    mask = s.problem.mask
    u_cp, _, _ = cp.run(s.A, s.At, s.b, s.cb, mask, s.lam_t, 8, 20000, 0.32, 0.32)
    st = pdrq.zero_state(s)
    for _ in range(3000):
        st = pdrq.step(s, st)
    assert np.max(np.abs(st.u - u_cp)) < 1e-8
