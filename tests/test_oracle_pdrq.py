"""Pins of the oracle's PDRQS1 iteration (thesis §4.4), setup (§5.1) and gap
record: optimality conditions derived from the problem (C_h), an independent
solver (Algorithm CP, §3.4), and special cases with textbook answers."""
import math

import numpy as np
import pytest

from oracle import cp, gap, geometry, pdrq, radon, tv


def _dense_ops(g):
    R = radon.radon_matrix(g)
    fwd = lambda u: (R @ u.ravel()).reshape(g.n_angles, g.n_bins)
    adj = lambda v: (R.T @ v.ravel()).reshape(g.n, g.n)
    return R, fwd, adj


@pytest.fixture(scope="module")
def tiny_metal():
    """8x8 image, 12 angles, 16 bins (R_h injective), one metal pixel whose
    trace is the constraint set D0; the bound C = R_h(tissue + 2 metal) on D0
    exceeds what the tissue data suggests, so the inequality is active."""
    g = geometry.Geometry(8, 12, 16)
    R, fwd, adj = _dense_ops(g)
    assert np.linalg.matrix_rank(R) == 64
    rng = np.random.default_rng(0)
    ut = np.zeros((8, 8))
    ut[2:6, 3:7] = 1.0
    metal = np.zeros((8, 8))
    metal[4, 4] = 1.0
    mask = fwd(metal) > 0
    u0 = fwd(ut) + 0.05 * rng.standard_normal((12, 16))
    prob = pdrq.Problem(g, u0, mask, fwd(ut + 2.0 * metal), lam=0.5)
    s = pdrq.setup(prob, pdrq.Params(), rng.standard_normal((8, 8)), rng.standard_normal((8, 8)),
                   fwd=fwd, adj=adj)
    st = pdrq.zero_state(s)
    for _ in range(10000):
        prev = st.u
        st, y1, w = pdrq.step(s, st, return_dual=True)
    return s, st, y1, w, prev, R


def test_normalization_uses_operator_norm(tiny_metal):
    """beta = ||R_h|| (power iteration, 30 steps) so that ||A|| ~ 1 (§5.1)."""
    s, *_, R = tiny_metal
    smax = np.linalg.svd(R, compute_uv=False)[0]
    assert s.beta == pytest.approx(smax, rel=1e-3)
    assert s.beta <= smax * (1 + 1e-12)
    assert s.lam_t == pytest.approx(0.5 / s.beta ** 2)


def test_kkt_conditions_at_convergence(tiny_metal):
    """Optimality of (C_h) (primal-dual system of §4.1 with the conjugates of
    §3.3): y1 = A u - b off D0; y1 <= 0, A u >= C~ and y1 (A u - C~) = 0 on D0;
    |w| <= lambda~/tau with w = (lambda~/tau) grad u/|grad u| where grad u != 0;
    A^* y1 - tau div w = 0."""
    s, st, y1, w, prev, _ = tiny_metal
    tau = s.params.tau
    mask = s.problem.mask
    Au = s.A(st.u)
    assert np.max(np.abs((y1 - (Au - s.b))[~mask])) < 1e-10
    assert np.all(y1[mask] <= 1e-12)
    assert np.all(Au[mask] >= s.cb[mask] - 1e-10)
    assert np.max(np.abs(y1[mask] * (Au[mask] - s.cb[mask]))) < 1e-10
    gu = tv.grad(st.u)
    ng = np.hypot(gu[0], gu[1])
    nw = np.hypot(w[0], w[1])
    assert np.all(nw <= s.lam_t / tau * (1 + 1e-12))
    act = ng > 1e-6
    assert act.sum() > 5
    assert np.max(np.abs(w[:, act] - s.lam_t / tau * gu[:, act] / ng[act])) < 1e-8
    assert np.max(np.abs(s.At(y1) - tau * tv.div(w))) < 1e-10
    rec = gap.record(s, st.u, y1, w, prev)
    assert abs(rec[2]) < 1e-10 and rec[3] < 1e-10 and rec[4] < 1e-10 and rec[5] < 1e-12
    # the constraint is active somewhere: the inequality matters
    assert np.any(np.abs(Au[mask] - s.cb[mask]) < 1e-8)


def test_fixed_point(tiny_metal):
    """A converged state is a fixed point of the iteration."""
    s, st, *_ = tiny_metal
    nxt = pdrq.step(s, st)
    assert np.max(np.abs(nxt.u - st.u)) < 1e-12
    assert np.max(np.abs(nxt.vb1 - st.vb1)) < 1e-12
    assert np.max(np.abs(nxt.vb2 - st.vb2)) < 1e-12


def test_cp_reaches_same_minimizer(tiny_metal):
    """Algorithm CP (§3.4), an unpreconditioned method with different steps,
    reaches the same u* (R_h injective, so the minimizer is unique)."""
    s, st, *_ = tiny_metal
    u, v, w = cp.run(s.A, s.At, s.b, s.cb, s.problem.mask, s.lam_t, 8, 20000, 0.32, 0.32)
    assert np.max(np.abs(u - st.u)) < 1e-9


def test_least_squares_special_case():
    """lambda = 0 and D0 empty: (P_h) is least squares; its minimizer is
    numpy.linalg.lstsq on the explicit matrix (well-conditioned 4x4 case;
    tau, which does not change the minimizer when lambda = 0, is taken small
    so that the Laplacian term of M does not slow the fit)."""
    g = geometry.Geometry(4, 16, 7)
    R, fwd, adj = _dense_ops(g)
    rng = np.random.default_rng(1)
    u0 = fwd(rng.uniform(0, 1, (4, 4))) + 0.1 * rng.standard_normal((16, 7))
    prob = pdrq.Problem(g, u0, np.zeros((16, 7), bool), np.zeros((16, 7)), lam=0.0)
    s = pdrq.setup(prob, pdrq.Params(tau=0.05), rng.standard_normal((4, 4)),
                   rng.standard_normal((4, 4)), fwd=fwd, adj=adj)
    st = pdrq.run(s, 4000)
    ls = np.linalg.lstsq(R, u0.ravel(), rcond=None)[0].reshape(4, 4)
    assert np.max(np.abs(st.u - ls)) < 1e-9


def test_huge_lambda_gives_constant(tiny_metal):
    """lambda -> infinity, D0 empty: TV forces a constant (nabla_h u = 0 iff u
    constant, §3.1) and the constant is the least-squares fit
    c* = <R_h 1, u0> / ||R_h 1||^2."""
    s0, *_, R = tiny_metal
    g = s0.problem.geom
    prob = pdrq.Problem(g, s0.problem.u0, np.zeros_like(s0.problem.mask), s0.problem.bound, lam=1e8)
    s = pdrq.setup(prob, pdrq.Params(), beta=s0.beta, c=s0.c, fwd=s0.fwd, adj=s0.adj)
    st = pdrq.run(s, 3000)
    one = (R @ np.ones(64))
    cstar = one @ s0.problem.u0.ravel() / (one @ one)
    assert np.max(np.abs(st.u - cstar)) < 1e-10


def test_fenchel_young_bound_of_gap_record(tiny_metal):
    """For any feasible u (A u >= C~ on D0) and dual-feasible y (y1 <= 0 on D0,
    |w| <= lambda~/tau): gap(u, y) - <u, K^* y> = G(Ku) + G^*(y) - <Ku, y> >= 0
    (Fenchel-Young); pins the signs and terms of the record."""
    s, st, *_ = tiny_metal
    rng = np.random.default_rng(2)
    tau = s.params.tau
    mask = s.problem.mask
    worst = np.inf
    for _ in range(200):
        u = st.u + 0.3 * rng.standard_normal(st.u.shape) + 0.5
        if not np.all(s.A(u)[mask] >= s.cb[mask]):
            continue
        y1 = rng.standard_normal(s.b.shape)
        y1[mask] = -np.abs(y1[mask])
        w = rng.standard_normal((2, 8, 8))
        nw = np.hypot(w[0], w[1])
        w = w / np.maximum(1, nw / (s.lam_t / tau)) * rng.uniform(0, 1, (8, 8))
        rec = gap.record(s, u, y1, w)
        kty = s.At(y1) - tau * tv.div(w)
        worst = min(worst, rec[2] - np.sum(u * kty))
    assert worst >= -1e-12 and np.isfinite(worst)


def test_gap_record_detects_flipped_sign(monkeypatch, tiny_metal):
    """Planting a sign error in the conjugate (y1 b -> -y1 b) in the oracle
    makes the Fenchel-Young pin fail: the pin has teeth."""
    s, st, y1, w, prev, _ = tiny_metal
    base = gap.record(s, st.u, y1, w, prev)
    bad_b = -s.b
    s2 = pdrq.Setup(s.problem, s.params, s.beta, s.c, bad_b, s.cb, s.lam_t, s.mult, s.fwd, s.adj)
    rec = gap.record(s2, st.u, y1, w, prev)
    assert abs(rec[2]) > 1e3 * max(abs(base[2]), 1e-14)


def test_nonneg_variant_matches_projected_cp(tiny_metal):
    """The u >= 0 variant (§4.5) reaches the minimizer of (C_h) + I{u >= 0},
    checked against Algorithm CP with the resolvent of F = I{u >= 0}."""
    s, *_ = tiny_metal
    g = s.problem.geom
    # make non-negativity active: data from an image with a negative dip
    R, fwd, adj = _dense_ops(g)
    ut = np.zeros((8, 8))
    ut[2:6, 3:7] = 1.0
    ut[1, 1] = -1.5
    prob = pdrq.Problem(g, fwd(ut), np.zeros((12, 16), bool), np.zeros((12, 16)), lam=0.2)
    sp = pdrq.setup(prob, pdrq.Params(), beta=s.beta, c=s.c, fwd=fwd, adj=adj)
    st = pdrq.zero_state_nonneg(sp)
    for _ in range(6000):
        st = pdrq.step_nonneg(sp, st)
    # projected CP
    u = np.zeros((8, 8)); ub = u.copy(); v = np.zeros((12, 16)); w = np.zeros((2, 8, 8))
    sig = t = 0.32
    from oracle import prox
    for _ in range(20000):
        w = prox.tv_project(w + t * tv.grad(ub), sp.lam_t)
        v = prox.prox_sino(v + t * sp.A(ub), t, sp.b, sp.cb, prob.mask)
        un = np.maximum(u + sig * tv.div(w) - sig * sp.At(v), 0.0)
        ub = 2 * un - u
        u = un
    assert np.min(st.u) > -1e-10
    assert np.max(np.abs(st.u - u)) < 1e-7
    assert np.min(u) == 0.0          # the constraint is active
