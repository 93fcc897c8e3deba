"""Pins of the oracle's ADMM (§4.6, no GPU): the soft thresholding satisfies
the optimality conditions of its minimization and beats a brute-force grid,
PCG solves the normal equation that a dense solve gives, and ADMM (exact and
one-step inner solves) reaches the minimizer that Algorithm CP reaches on a
tiny injective problem, with z = K u at the limit."""
import numpy as np
import pytest

from oracle import admm, cp, geometry, pdrq, radon, tv


def test_soft_threshold_optimality():
    rng = np.random.default_rng(0)
    q = rng.standard_normal((2, 40, 1)) * 2.0
    t = 1.3
    x = admm.soft_threshold(q, t)
    nq = np.hypot(q[0], q[1])[:, 0]
    nx = np.hypot(x[0], x[1])[:, 0]
    for k in range(40):
        if nq[k] <= t:
            # 0 is optimal iff q lies in the subdifferential t * (unit ball)
            assert nx[k] == 0.0
        else:
            # x != 0 and x - q + t x / |x| = 0
            g = x[:, k, 0] - q[:, k, 0] + t * x[:, k, 0] / nx[k]
            assert nx[k] > 0 and np.max(np.abs(g)) < 1e-12


def test_soft_threshold_beats_grid():
    rng = np.random.default_rng(1)
    t = 0.7
    xs = np.linspace(-3, 3, 601)
    X, Y = np.meshgrid(xs, xs)
    for _ in range(5):
        q = rng.standard_normal(2) * 1.5
        f = 0.5 * ((X - q[0]) ** 2 + (Y - q[1]) ** 2) + t * np.hypot(X, Y)
        x = admm.soft_threshold(q.reshape(2, 1, 1), t).ravel()
        fx = 0.5 * np.sum((x - q) ** 2) + t * np.hypot(*x)
        assert fx <= f.min() + 1e-12


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
                   fwd=fwd, adj=adj)
    return s, R


def test_pcg_solves_the_normal_equation(tiny):
    s, R = tiny
    n = s.problem.geom.n
    tau = s.params.tau
    # dense H = A^T A - tau^2 div grad from its action on unit images
    cols = []
    for k in range(n * n):
        e = np.zeros(n * n)
        e[k] = 1.0
        cols.append(admm.H(s, e.reshape(n, n)).ravel())
    Hd = np.array(cols).T
    A = R / s.beta
    G = np.array([tv.grad(np.eye(n * n)[k].reshape(n, n), 1.0).ravel() for k in range(n * n)]).T
    assert np.allclose(Hd, A.T @ A + tau * tau * G.T @ G, atol=1e-12)
    rng = np.random.default_rng(3)
    rhs = rng.standard_normal((n, n))
    want = np.linalg.solve(Hd, rhs.ravel()).reshape(n, n)
    mult = admm.multiplier_admm(n, tau, s.c, s.params.eps)
    got = admm.pcg(s, rhs, np.zeros((n, n)), 200, mult)
    assert np.max(np.abs(got - want)) < 1e-9 * max(1.0, np.max(np.abs(want)))
    # one step from the solution stays there (zero residual: alpha = 0)
    again = admm.pcg(s, rhs, want, 1, mult)
    assert np.max(np.abs(again - want)) < 1e-9


@pytest.mark.parametrize("cg_steps,iters", [(60, 3000), (1, 6000)])
def test_admm_reaches_the_cp_minimizer(tiny, cg_steps, iters):
    s, _ = tiny
    mask = s.problem.mask
    u_cp, _, _ = cp.run(s.A, s.At, s.b, s.cb, mask, s.lam_t, 8, 20000, 0.32, 0.32)
    st = admm.run(s, iters, cg_steps)
    assert np.max(np.abs(st.u - u_cp)) < 1e-6
    # primal feasibility at the limit: z = K u
    assert np.max(np.abs(st.zw - s.A(st.u))) < 1e-6
    assert np.max(np.abs(st.zv - tv.grad(st.u, 1.0))) < 1e-6
