"""Pins of the PDRQ3 splitting (§4.4, table of splittings; no GPU): on a tiny
injective problem with an active constraint it reaches the minimizer that
Algorithm CP reaches, its duals satisfy the optimality conditions of (C_h),
and the minimizer is a fixed point of its iteration."""
import numpy as np
import pytest

from oracle import cp, geometry, pdrq, pdrq3, radon, tv


@pytest.fixture(scope="module")
def tiny_metal3():
    g = geometry.Geometry(8, 12, 16)
    R = radon.radon_matrix(g)
    fwd = lambda u: (R @ u.ravel()).reshape(g.n_angles, g.n_bins)
    adj = lambda v: (R.T @ v.ravel()).reshape(g.n, g.n)
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
    st = pdrq3.run3(s, 10000)
    return s, st


def test_pdrq3_reaches_the_cp_minimizer(tiny_metal3):
    s, st = tiny_metal3
    u_cp, _, _ = cp.run(s.A, s.At, s.b, s.cb, s.problem.mask, s.lam_t, 8, 40000, 0.32, 0.32)
    assert np.max(np.abs(st.u - u_cp)) < 1e-7
    # the inequality is active somewhere (A u = C~ on part of D0)
    mask = s.problem.mask
    r = s.A(st.u)
    assert np.any(np.abs(r - s.cb)[mask] < 1e-6)
    assert np.all(r[mask] >= s.cb[mask] - 1e-7)


def test_pdrq3_duals_satisfy_optimality(tiny_metal3):
    # at the fixed point the data dual is v1: vb1 itself off D0 (there the
    # resolvent is the identity), vb1 + sigma A u on D0 (the resolvent's fixed
    # point); it is A u - b off D0, <= 0 with complementarity on D0, and
    # A^* y1 - tau div w = 0 for the TV dual w = the projected 2 v2 - vb2
    s, st = tiny_metal3
    mask = s.problem.mask
    tau, sig = s.params.tau, s.params.sigma
    r = s.A(st.u)
    y1 = np.where(mask, st.vb1 + sig * r, st.vb1)
    assert np.max(np.abs((y1 - (r - s.b))[~mask])) < 1e-7
    assert np.all(y1[mask] <= 1e-9)
    assert np.max(np.abs(y1[mask] * (r - s.cb)[mask])) < 1e-8
    g = tv.grad(st.u, 1.0)
    v2 = st.vb2 + sig * tau * g
    from oracle import prox
    w = prox.tv_project(2.0 * v2 - st.vb2, s.lam_t / tau)
    assert np.max(np.abs(s.At(y1) - tau * tv.div(w, 1.0))) < 1e-7


def test_pdrq3_fixed_point(tiny_metal3):
    s, st = tiny_metal3
    nxt = pdrq3.step3(s, st)
    assert np.max(np.abs(nxt.u - st.u)) < 1e-10
    assert np.max(np.abs(nxt.vb1 - st.vb1)) < 1e-10
