"""Pins of the oracle's reverse-mode derivative of unrolled PDRQS1 (no GPU):
central finite differences of the unrolled map itself, in lambda and along
random directions of the data u0, on small problems with and without a metal
trace.  beta and c are fixed so that the map u0, lambda -> u_K is exactly the
composition of K iterations."""
import numpy as np
import pytest

from oracle import geometry, pdrq, radon, unrolled


def small_problem(seed, metal):
    rng = np.random.default_rng(seed)
    n, N, M = 12, 20, 18
    g = geometry.Geometry(n, N, M)
    truth = np.zeros((n, n))
    truth[3:9, 2:8] = 1.0
    truth[5:7, 6:10] += 0.5
    u0 = radon.radon_fwd(g, truth) + 0.05 * rng.standard_normal((N, M))
    if metal:
        blob = np.zeros((n, n))
        blob[5:7, 5:7] = 1.0
        mask = radon.radon_fwd(g, blob) > 0.5
        bound = np.where(mask, 0.9 * radon.radon_fwd(g, truth), 0.0)
    else:
        mask = np.zeros((N, M), dtype=bool)
        bound = np.zeros((N, M))
    return g, truth, u0, mask, bound


def estimate_beta_c(g, u0, mask, bound, lam):
    rng = np.random.default_rng(1)
    s0 = pdrq.setup(pdrq.Problem(g, u0, mask, bound, lam), pdrq.Params(),
                    rng.standard_normal((g.n, g.n)), rng.standard_normal((g.n, g.n)))
    return s0.beta, s0.c


def unrolled_loss(g, truth, u0, mask, bound, lam, K, beta, c):
    s = pdrq.setup(pdrq.Problem(g, u0, mask, bound, lam), pdrq.Params(), beta=beta, c=c)
    states = unrolled.forward(s, K)
    L, gbar = unrolled.mse_loss(states[-1].u, truth)
    return L, gbar, s, states


@pytest.mark.parametrize("metal", [False, True])
def test_gradients_match_finite_differences(metal):
    g, truth, u0, mask, bound = small_problem(7, metal)
    lam, K = 0.3, 15
    beta, c = estimate_beta_c(g, u0, mask, bound, lam)
    L, gbar, s, states = unrolled_loss(g, truth, u0, mask, bound, lam, K, beta, c)
    du0, dlam = unrolled.backward(s, states, gbar)
    # lambda
    d = 1e-5 * lam
    Lp = unrolled_loss(g, truth, u0, mask, bound, lam + d, K, beta, c)[0]
    Lm = unrolled_loss(g, truth, u0, mask, bound, lam - d, K, beta, c)[0]
    fd = (Lp - Lm) / (2 * d)
    assert dlam == pytest.approx(fd, rel=1e-5, abs=1e-12)
    assert abs(dlam) > 1e-8
    # u0 along random directions
    rng = np.random.default_rng(11)
    for _ in range(3):
        v = rng.standard_normal(u0.shape)
        e = 1e-5
        Lp = unrolled_loss(g, truth, u0 + e * v, mask, bound, lam, K, beta, c)[0]
        Lm = unrolled_loss(g, truth, u0 - e * v, mask, bound, lam, K, beta, c)[0]
        fd = (Lp - Lm) / (2 * e)
        an = float(np.sum(du0 * v))
        assert an == pytest.approx(fd, rel=1e-5, abs=1e-12)
    # the data on the metal trace does not enter (the bound replaces it there)
    if metal:
        assert np.all(du0[mask] == 0.0)


def test_gradient_of_one_iteration_is_linear_algebra():
    """K = 1 from the zero state: u_1 = M^{-1}(0) = 0, so dL/du0 and dL/dlambda
    vanish; K = 2 has a nonzero data gradient but still none in lambda (w of
    the first iteration is the projection of 0)."""
    g, truth, u0, mask, bound = small_problem(3, False)
    for K, lam_zero in ((1, True), (2, True)):
        s = pdrq.setup(pdrq.Problem(g, u0, mask, bound, 0.3), pdrq.Params(), beta=20.0, c=2.0)
        states = unrolled.forward(s, K)
        _, gbar = unrolled.mse_loss(states[-1].u, truth)
        du0, dlam = unrolled.backward(s, states, gbar)
        assert dlam == 0.0
        if K == 1:
            assert np.all(du0 == 0.0)
        else:
            assert np.abs(du0).max() > 0


def test_planted_sign_error_fails_fd():
    """A flipped sign in the gradient-side adjoint (a plausible mistake) is
    caught by the finite-difference check."""
    g, truth, u0, mask, bound = small_problem(7, False)
    lam, K = 0.3, 10
    beta, c = estimate_beta_c(g, u0, mask, bound, lam)
    L, gbar, s, states = unrolled_loss(g, truth, u0, mask, bound, lam, K, beta, c)
    orig = unrolled.tv.div
    try:
        unrolled.tv.div = lambda p, h: -orig(p, h)
        _, dlam_bad = unrolled.backward(s, states, gbar)
    finally:
        unrolled.tv.div = orig
    d = 1e-5 * lam
    fd = (unrolled_loss(g, truth, u0, mask, bound, lam + d, K, beta, c)[0]
          - unrolled_loss(g, truth, u0, mask, bound, lam - d, K, beta, c)[0]) / (2 * d)
    assert abs(dlam_bad - fd) > 1e-3 * abs(fd)
