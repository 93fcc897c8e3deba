"""Pins of the comparison methods of the oracle (no GPU): PDRQS2 (§4.2,
§4.3.1) and PDRQS1 with the Richardson preconditioner (§4.3) reach the
minimizer that Algorithm CP (§3.4) and PDRQS1 reach on a tiny injective
unconstrained problem, their fixed points are those minimizers, and the
objective helper reproduces hand-computed values."""
import numpy as np
import pytest

from oracle import cp, geometry, pdrq, pdrq2, radon, tv


@pytest.fixture(scope="module")
def tiny_free():
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
    u_cp, _, _ = cp.run(s.A, s.At, s.b, s.cb, mask, s.lam_t, 8, 20000, 0.32, 0.32)
    return s, u_cp


def test_pdrqs2_reaches_the_minimizer(tiny_free):
    s, u_cp = tiny_free
    st = pdrq2.zero_state2(s)
    for _ in range(4000):
        st = pdrq2.step2(s, st)
    assert np.max(np.abs(st.u - u_cp)) < 1e-8
    # a fixed point of the iteration
    nxt = pdrq2.step2(s, st)
    assert np.max(np.abs(nxt.u - st.u)) < 1e-12
    assert np.max(np.abs(nxt.vb - st.vb)) < 1e-12


def test_richardson_reaches_the_minimizer(tiny_free):
    s, u_cp = tiny_free
    sr = pdrq2.richardson_setup(s)
    st = pdrq.zero_state(sr)
    for _ in range(20000):
        st = pdrq.step(sr, st)
    assert np.max(np.abs(st.u - u_cp)) < 1e-8


def test_inverse_norm_preconditioning_beats_richardson(tiny_free):
    """The point of §4.3.1 on a small case: after the same number of
    iterations the inverse-norm preconditioned PDRQS1 is much closer to the
    minimizer than the Richardson choice."""
    s, u_cp = tiny_free
    sr = pdrq2.richardson_setup(s)
    a, b = pdrq.zero_state(s), pdrq.zero_state(sr)
    for _ in range(200):
        a, b = pdrq.step(s, a), pdrq.step(sr, b)
    assert np.linalg.norm(a.u - u_cp) < 0.1 * np.linalg.norm(b.u - u_cp)


def test_objective_by_hand():
    g = geometry.Geometry(6, 5, 9)
    rng = np.random.default_rng(3)
    u0 = rng.standard_normal((5, 9))
    mask = np.zeros((5, 9), dtype=bool)
    mask[1, 2:5] = True
    bound = np.where(mask, 2.0, 0.0)
    s = pdrq.setup(pdrq.Problem(g, u0, mask, bound, 0.7), pdrq.Params(), beta=3.0, c=1.0)
    fit, reg, viol = pdrq2.objective(s, np.zeros((6, 6)))
    assert fit == pytest.approx(0.5 * np.sum(u0[~mask] ** 2))
    assert reg == 0.0 and viol == 2.0
    u = np.zeros((6, 6))
    u[2, 3] = 1.0
    fit, reg, viol = pdrq2.objective(s, u)
    r = radon.radon_fwd(g, u)
    assert fit == pytest.approx(0.5 * np.sum((r - u0)[~mask] ** 2))
    # an isolated pixel: forward differences give |grad u| = sqrt(2) at the
    # pixel and 1 at its left and upper neighbours
    assert reg == pytest.approx(0.7 * (np.sqrt(2.0) + 2.0))
    assert viol == pytest.approx(np.max(2.0 - r[mask]))


@pytest.fixture(scope="module")
def tiny_metal_clean():
    """8x8, 12 angles, 16 bins, noise-free data (so that the hard constraint
    A u = b off D0 is feasible), one metal pixel whose trace is D0."""
    g = geometry.Geometry(8, 12, 16)
    R = radon.radon_matrix(g)
    fwd = lambda u: (R @ u.ravel()).reshape(g.n_angles, g.n_bins)
    adj = lambda v: (R.T @ v.ravel()).reshape(g.n, g.n)
    rng = np.random.default_rng(4)
    ut = np.zeros((8, 8))
    ut[2:6, 3:7] = 1.0
    metal = np.zeros((8, 8))
    metal[4, 4] = 1.0
    mask = fwd(metal) > 0
    u0 = np.where(mask, fwd(ut + 3.0 * metal), fwd(ut))
    prob = pdrq.Problem(g, u0, mask, 0.9 * fwd(ut), lam=0.2)
    s = pdrq.setup(prob, pdrq.Params(), rng.standard_normal((8, 8)), rng.standard_normal((8, 8)),
                   fwd=fwd, adj=adj)
    return s


@pytest.mark.parametrize("fit", ["weighted", "ignore", "everywhere", "hard"])
def test_data_term_variants_reach_the_cp_minimizer(tiny_metal_clean, fit):
    """Each data-term variant of §3.5 in PDRQS1 reaches the minimizer that
    Algorithm CP reaches with the same resolvent (two different iterations,
    one answer; the resolvents themselves are pinned against scipy)."""
    import dataclasses
    s = dataclasses.replace(tiny_metal_clean, fit=fit)
    if fit == "weighted":
        s = dataclasses.replace(s, weight=np.linspace(0.5, 2.0, s.b.size).reshape(s.b.shape))
    st = pdrq.zero_state(s)
    for _ in range(15000):
        st = pdrq.step(s, st)
    res = lambda q, step: pdrq.sino_resolvent(s, q, step)
    u_cp, _, _ = cp.run(s.A, s.At, s.b, s.cb, s.problem.mask, s.lam_t, 8, 30000, 0.32, 0.32,
                        resolvent=res)
    assert np.max(np.abs(st.u - u_cp)) < 1e-6
    if fit == "hard":
        r = s.A(st.u)
        assert np.max(np.abs((r - s.b)[~s.problem.mask])) < 1e-6


def test_variant_identities(tiny_metal_clean):
    """Weights of 1 are the standard fit; ignoring D0 is the standard fit with
    an unreachable bound C~ -> -infinity."""
    import dataclasses
    s = tiny_metal_clean
    q = np.random.default_rng(9).standard_normal(s.b.shape)
    std = pdrq.sino_resolvent(s, q, 0.7)
    w1 = pdrq.sino_resolvent(dataclasses.replace(s, fit="weighted"), q, 0.7)
    assert np.array_equal(std, w1)
    ign = pdrq.sino_resolvent(dataclasses.replace(s, fit="ignore"), q, 0.7)
    low = pdrq.sino_resolvent(dataclasses.replace(s, cb=np.full_like(s.cb, -1e30)), q, 0.7)
    assert np.array_equal(ign, low)
