"""The comparison methods on the GPU against the FP64 oracle: PDRQS1 with the
Richardson preconditioner (§4.3), Algorithm CP (§3.4), PDRQS2 (§4.2, §4.3.1),
and the objective of (C_h)."""
import numpy as np
import pytest
import torch

import synth
from oracle import admm, cp, pdrq, pdrq2, tv

from oracle_inputs import build, f32

pytestmark = pytest.mark.gpu

ct = pytest.importorskip("paper_1810_03275_amd")

DEV = torch.device("cuda")


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def gpu(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(DEV)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def _metal(n=64, N=90, M=96):
    w = synth.workload("C2", n=n, n_angles=N, n_bins=M)
    g, u0, mask, bound = build(w)
    return w, g, u0, mask, bound


def _free(n=64, N=90, M=96):
    w = synth.workload("C1", n=n, n_angles=N, n_bins=M)
    g, u0, mask, bound = build(w)
    assert not mask.any()
    return w, g, u0, mask, bound


def test_objective_matches_oracle():
    print("objective", flush=True)
    w, g, u0, mask, bound = _metal()
    plan = ct.Plan(g.n, g.n_angles, g.n_bins)
    u = f32(np.random.default_rng(5).uniform(-0.5, 1.0, (g.n, g.n)))
    got = ct.objective(plan, gpu(u0), w.alpha, gpu(u), ct.pack_mask(mask), gpu(bound))
    s = pdrq.setup(pdrq.Problem(g, u0, mask, bound, w.alpha), pdrq.Params(), beta=1.0, c=1.0)
    fit, reg, viol = pdrq2.objective(s, u)
    assert got[0] == pytest.approx(fit, rel=1e-5)
    assert got[1] == pytest.approx(reg, rel=1e-5)
    assert got[2] == pytest.approx(viol, rel=1e-4, abs=1e-5 * max(1.0, viol))


def test_richardson_matches_oracle():
    print("richardson", flush=True)
    w, g, u0, mask, bound = _metal()
    plan = ct.Plan(g.n, g.n_angles, g.n_bins)
    mb = ct.pack_mask(mask)
    probe = ct.Solver(plan, gpu(u0), w.alpha, mb, gpu(bound))
    inf = probe.info()
    u, _ = ct.reconstruct(plan, gpu(u0), w.alpha, mb, gpu(bound), k_max=60, beta=inf["beta"],
                          c=inf["c"], method="richardson")
    s = pdrq.setup(pdrq.Problem(g, u0, mask, bound, w.alpha), pdrq.Params(), beta=inf["beta"],
                   c=inf["c"])
    sr = pdrq2.richardson_setup(s)
    st = pdrq.zero_state(sr)
    for _ in range(60):
        st = pdrq.step(sr, st)
    assert rel(host(u), st.u) <= 1e-4


def test_cp_matches_oracle():
    print("cp", flush=True)
    w, g, u0, mask, bound = _metal()
    plan = ct.Plan(g.n, g.n_angles, g.n_bins)
    mb = ct.pack_mask(mask)
    probe = ct.Solver(plan, gpu(u0), w.alpha, mb, gpu(bound))
    inf = probe.info()
    u, _ = ct.reconstruct(plan, gpu(u0), w.alpha, mb, gpu(bound), k_max=100, beta=inf["beta"],
                          c=inf["c"], method="cp")
    s = pdrq.setup(pdrq.Problem(g, u0, mask, bound, w.alpha), pdrq.Params(), beta=inf["beta"],
                   c=inf["c"])
    step = 0.99 / 3.0
    uo, _, _ = cp.run(s.A, s.At, s.b, s.cb, mask, s.lam_t, g.n, 100, step, step)
    assert rel(host(u), uo) <= 1e-4


def test_pdrqs2_matches_oracle():
    print("pdrqs2", flush=True)
    w, g, u0, mask, bound = _free()
    plan = ct.Plan(g.n, g.n_angles, g.n_bins)
    probe = ct.Solver(plan, gpu(u0), w.alpha)
    inf = probe.info()
    sv = ct.Solver(plan, gpu(u0), w.alpha, beta=inf["beta"], c=inf["c"], method="pdrqs2")
    sv.step(100)
    s = pdrq.setup(pdrq.Problem(g, u0, mask, bound, w.alpha), pdrq.Params(), beta=inf["beta"],
                   c=inf["c"])
    st = pdrq2.zero_state2(s)
    for _ in range(100):
        st = pdrq2.step2(s, st)
    assert rel(host(sv.export()[0]), st.u) <= 1e-4
    # one step from an imported random state
    rng = np.random.default_rng(8)
    u = f32(rng.uniform(0, 1, (g.n, g.n)))
    vb = f32(s.lam_t / s.params.tau * rng.standard_normal((2, g.n, g.n)))
    sv.import_state(gpu(u), torch.zeros((g.n_angles, g.n_bins), device=DEV), gpu(vb))
    sv.step(1)
    nxt = pdrq2.step2(s, pdrq2.State2(u, vb))
    gu, _, gvb = (host(t) for t in sv.export())
    assert rel(gu, nxt.u) <= 1e-5
    assert rel(gvb, nxt.vb) <= 1e-5


def test_method_errors():
    plan = ct.Plan(32, 45, 48)
    z = torch.zeros((45, 48), device=DEV)
    m = ct.pack_mask(np.ones((45, 48), dtype=bool))
    with pytest.raises(ct.CtpdError):
        ct.Solver(plan, z, 0.01, m, method="pdrqs2")     # PDRQS2 has no D0
    with pytest.raises(ct.CtpdError):
        ct.Solver(plan, z, 0.01, method="cp", nonneg=True)
    with pytest.raises(ValueError):
        ct.Solver(plan, z, 0.01, method="no-such-method")
    with pytest.raises(ct.CtpdError):
        ct.Solver(plan, z, 0.01, m, method="admm")       # ADMM has no D0
    with pytest.raises(ct.CtpdError):
        ct.Solver(plan, z, 0.01, method="admm", cg_steps=0)
    with pytest.raises(ct.CtpdError):
        ct.Solver(plan, z, 0.01, method="admm", mu=-1.0)
    sa = ct.Solver(plan, z, 0.01, method="admm")
    sa.step(1)
    assert ct.lib.ct_solver_set_admm(sa._h, 2, 1.0) != 0  # after the first iteration
    with pytest.raises(ct.CtpdError):
        sa.gap()
    sv = ct.Solver(plan, z, 0.01, method="cp")
    sv.step(2)
    with pytest.raises(ct.CtpdError):
        sv.gap()


@pytest.mark.parametrize("cg_steps,mu", [(1, 1.0), (2, 1.0), (1, 2.0)])
def test_admm_matches_oracle(cg_steps, mu):
    print("admm", cg_steps, mu, flush=True)
    w, g, u0, mask, bound = _free()
    plan = ct.Plan(g.n, g.n_angles, g.n_bins)
    probe = ct.Solver(plan, gpu(u0), w.alpha)
    inf = probe.info()
    s = pdrq.setup(pdrq.Problem(g, u0, mask, bound, w.alpha), pdrq.Params(), beta=inf["beta"],
                   c=inf["c"])
    st = admm.zero_state(s)
    done = 0
    for k, tol in ((1, 1e-5), (2, 1e-5), (3, 1e-5), (40, 1e-4)):
        sv = ct.Solver(plan, gpu(u0), w.alpha, beta=inf["beta"], c=inf["c"], method="admm",
                       cg_steps=cg_steps, mu=mu)
        sv.step(k)
        while done < k:
            st = admm.step(s, st, cg_steps, mu)
            done += 1
        gu, gew, gev = (host(t) for t in sv.export())
        assert rel(gu, st.u) <= tol, (k, rel(gu, st.u))
        # the multipliers are small differences of the projections and
        # gradients they are formed from (eta_v lies in the ball of radius
        # lambda~/(mu tau^2)), so their FP32 error is measured on that scale
        sw = max(np.linalg.norm(s.A(st.u)), np.linalg.norm(st.ew))
        sv_ = max(np.linalg.norm(tv.grad(st.u, 1.0)), np.linalg.norm(st.ev))
        assert np.linalg.norm(gew - st.ew) <= 10 * tol * sw
        assert np.linalg.norm(gev - st.ev) <= 10 * tol * sv_


@pytest.mark.parametrize("kind", ["impulse", "circulant"])
def test_kernel_preconditioner_matches_oracle(kind):
    print("kernel preconditioner", kind, flush=True)
    w, g, u0, mask, bound = _metal()
    plan = ct.Plan(g.n, g.n_angles, g.n_bins)
    mb = ct.pack_mask(mask)
    sv = ct.Solver(plan, gpu(u0), w.alpha, mb, gpu(bound), precond=kind)
    inf = sv.info()
    # c from the oracle's own power iteration (another start vector)
    rng = np.random.default_rng(9)
    s_own = pdrq.setup(pdrq.Problem(g, u0, mask, bound, w.alpha), pdrq.Params(),
                       beta=inf["beta"], start_precond=rng.standard_normal((g.n, g.n)),
                       kind=kind)
    assert inf["c"] == pytest.approx(s_own.c, rel=0.05)
    s = pdrq.setup(pdrq.Problem(g, u0, mask, bound, w.alpha), pdrq.Params(), beta=inf["beta"],
                   c=inf["c"], kind=kind)
    st = pdrq.zero_state(s)
    done = 0
    for k, tol in ((1, 1e-5), (60, 1e-4)):
        sk = ct.Solver(plan, gpu(u0), w.alpha, mb, gpu(bound), precond=kind,
                       beta=inf["beta"], c=inf["c"])
        sk.step(k)
        while done < k:
            st = pdrq.step(s, st)
            done += 1
        assert rel(host(sk.export()[0]), st.u) <= tol


def test_kernel_preconditioner_errors():
    plan = ct.Plan(32, 45, 48)
    z = torch.zeros((45, 48), device=DEV)
    with pytest.raises(ct.CtpdError):
        ct.Solver(plan, z, 0.01, method="cp", precond="impulse")
    with pytest.raises(ct.CtpdError):
        ct.Solver(plan, z, 0.01, method="pdrqs2", precond="circulant")
    with pytest.raises(ct.CtpdError):
        ct.Solver(plan, z, 0.01, nonneg=True, precond="impulse")
    with pytest.raises(ValueError):
        ct.Solver(plan, z, 0.01, precond="no-such-preconditioner")


def test_pdrqs3_matches_oracle():
    print("pdrqs3", flush=True)
    from oracle import pdrq3
    w, g, u0, mask, bound = _metal()
    plan = ct.Plan(g.n, g.n_angles, g.n_bins)
    mb = ct.pack_mask(mask)
    probe = ct.Solver(plan, gpu(u0), w.alpha, mb, gpu(bound))
    inf = probe.info()
    s = pdrq.setup(pdrq.Problem(g, u0, mask, bound, w.alpha), pdrq.Params(), beta=inf["beta"],
                   c=inf["c"])
    st = pdrq.zero_state(s)
    done = 0
    # a plan of its own, so that the first PDRQS3 solver times its launch
    # choices on its own zero state (whose s1 is not zero) and the second
    # reuses them
    plan3 = ct.Plan(g.n, g.n_angles, g.n_bins)
    for k, tol in ((1, 1e-5), (60, 1e-4)):
        sv = ct.Solver(plan3, gpu(u0), w.alpha, mb, gpu(bound), beta=inf["beta"], c=inf["c"],
                       method="pdrqs3")
        assert sv.tuning()["source"] == ("timed" if k == 1 else "plan")
        sv.step(k)
        while done < k:
            st = pdrq3.step3(s, st)
            done += 1
        gu, gv1, gv2 = (host(t) for t in sv.export())
        assert rel(gu, st.u) <= tol
        assert rel(gv1, st.vb1) <= 10 * tol
    # one step from an imported random state (the cache rebuilt from it)
    rng = np.random.default_rng(12)
    u = f32(rng.uniform(0, 1, (g.n, g.n)))
    vb1 = f32(0.01 * rng.standard_normal((g.n_angles, g.n_bins)))
    vb2 = f32(s.lam_t / s.params.tau * rng.standard_normal((2, g.n, g.n)))
    sv.import_state(gpu(u), gpu(vb1), gpu(vb2))
    sv.step(1)
    nxt = pdrq3.step3(s, pdrq.state_from(s, u, vb1, vb2))
    gu, gv1, gv2 = (host(t) for t in sv.export())
    assert rel(gu, nxt.u) <= 1e-5
    assert rel(gv1, nxt.vb1) <= 1e-5
    assert rel(gv2, nxt.vb2) <= 1e-5
    with pytest.raises(ct.CtpdError):
        sv.gap()
