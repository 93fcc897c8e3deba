"""Batched PDRQS1 (many slices, uneven shapes) through the C ABI.

A batch advances every slice of one geometry with one launch per kernel, and
all batches of a solve replay as one HIP graph.  Each slice's result must be
the single-slice result (bitwise when both use the same backprojection
slicing) and match the FP64 oracle run with the same beta and c.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import pdrq

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


def small_batch(count, seed, sizes=(32, 48, 64)):
    shapes = synth.batched_shapes(count, seed=seed, sizes=sizes)
    out = []
    for i, sh in enumerate(shapes):
        w = synth.batched_workload(i, sh, iters=30)
        g, u0, mask, bound = build(w)
        out.append((w, g, u0, mask, bound))
    return out


NO_TUNE = ct.Launch(tune=False)


@pytest.mark.parametrize("kern", ["auto", "pairs8", "one_angle", "walk4"])
def test_batch_equals_single_slices(kern):
    """Three slices of one geometry in a batch solver vs three single solvers
    with the same launch choices: bitwise equal state after 25 iterations
    (same kernels, same order); also with R_h walking four angles at a time
    on a plan that walks two (forward tables of each solver's own)."""
    print("batch vs single", kern, flush=True)
    if kern == "walk4":
        launch = ct.Launch(tune=False, fwd_walk=4)
    else:
        launch = NO_TUNE if kern == "auto" else ct.Launch(tune=False, bp_kernel=kern)
    n, N, M = 64, 90, 96
    ws = [synth.batched_workload(i, (n, N, M, i % 3), iters=25) for i in range(3)]
    data = [build(w) for w in ws]
    plan = ct.Plan(n, N, M)
    sinos = [gpu(d[1]) for d in data]
    masks = [ct.pack_mask(d[2]) for d in data]
    bounds = [gpu(d[3]) for d in data]
    sb = ct.SolverBatch(plan, sinos, 0.005, masks, bounds, launch=launch)
    info = sb.info()
    assert sb.layout()["problems"] == 3
    if kern == "walk4":
        assert sb.layout()["angles_per_walk"] == 4 and plan.layout()["angles_per_walk"] == 2
    sb.step(25)
    ub, vb1b, vb2b = (host(t) for t in sb.export())
    gb = sb.gap()
    for b in range(3):
        sv = ct.Solver(plan, sinos[b], 0.005, masks[b], bounds[b], beta=info["beta"],
                       c=info["c"], launch=launch)
        sv.step(25)
        u, vb1, vb2 = (host(t) for t in sv.export())
        assert np.array_equal(u, ub[b])
        assert np.array_equal(vb1, vb1b[b])
        assert np.array_equal(vb2, vb2b[b])
        assert np.allclose(sv.gap(), gb[b], rtol=1e-12, atol=0)


def test_batch_state_roundtrip():
    """Export / import of a batch state restores the caches: continuing from an
    imported state gives the same iterates as continuing in place."""
    print("batch roundtrip", flush=True)
    n, N, M = 48, 67, 72
    ws = [synth.batched_workload(i, (n, N, M, 1), iters=10) for i in range(2)]
    data = [build(w) for w in ws]
    plan = ct.Plan(n, N, M)
    args = ([gpu(d[1]) for d in data], 0.005, [ct.pack_mask(d[2]) for d in data],
            [gpu(d[3]) for d in data])
    a = ct.SolverBatch(plan, *args)
    inf = a.info()
    b = ct.SolverBatch(plan, *args, beta=inf["beta"], c=inf["c"])
    a.step(7)
    b.import_state(*a.export())
    a.step(5)
    b.step(5)
    assert rel(host(a.export()[0]), host(b.export()[0])) <= 1e-6


def test_reconstruct_batched_uneven_vs_oracle():
    """Seven slices of three shapes (32, 48, 64 with N = 1.4 n, M = 1.5 n, 0-3
    metal discs) in one batched solve: every slice matches the oracle's 30
    iterations with the batch's beta and c to 1e-4, and the single-slice GPU
    solve to 1e-6."""
    print("batched uneven", flush=True)
    items = small_batch(7, seed=3100)
    plans = {}
    problems = []
    for w, g, u0, mask, bound in items:
        key = (g.n, g.n_angles, g.n_bins)
        if key not in plans:
            plans[key] = ct.Plan(*key)
        problems.append(dict(plan=plans[key], sino=gpu(u0), lam=w.alpha,
                             mask_bits=ct.pack_mask(mask), bound=gpu(bound)))
    us, rep = ct.reconstruct_batched(problems, k_max=30, gap_every=15)
    assert rep.shape == (7, 2, 6) and np.all(np.isfinite(rep))
    for (w, g, u0, mask, bound), pr, u in zip(items, problems, us):
        # beta and c of this geometry, as the batch estimated them
        probe = ct.Solver(pr["plan"], pr["sino"], w.alpha, pr["mask_bits"], pr["bound"])
        inf = probe.info()
        u1, _ = ct.reconstruct(pr["plan"], pr["sino"], w.alpha, pr["mask_bits"], pr["bound"],
                               k_max=30)
        assert rel(host(u), host(u1)) <= 1e-6
        s = pdrq.setup(pdrq.Problem(g, u0, mask, bound, w.alpha), pdrq.Params(),
                       beta=inf["beta"], c=inf["c"])
        st = pdrq.zero_state(s)
        for _ in range(30):
            st = pdrq.step(s, st)
        assert rel(host(u), st.u) <= 1e-4


def test_batched_groups_and_errors():
    """Two lambdas on one plan run as two batches; a negative lambda and an
    empty batch are rejected."""
    plan = ct.Plan(32, 45, 48)
    z = torch.zeros((45, 48), device=DEV)
    us, rep = ct.reconstruct_batched([dict(plan=plan, sino=z, lam=0.01),
                                      dict(plan=plan, sino=z, lam=0.02)], k_max=3)
    assert len(us) == 2 and rep is None
    assert all(float(u.abs().max()) == 0.0 for u in us)   # zero data: u stays 0
    with pytest.raises(ct.CtpdError):
        ct.SolverBatch(plan, [z, z], -1.0)
    with pytest.raises(ValueError):
        ct.SolverBatch(plan, [], 0.01)


def test_group_step_equals_separate_steps():
    """Two batches of different geometries stepped as one group (one graph)
    give bitwise the same state as stepping each batch on its own."""
    print("group step", flush=True)
    geo = [(48, 67, 72), (64, 90, 96)]
    made = []
    for gi, (n, N, M) in enumerate(geo):
        ws = [synth.batched_workload(10 * gi + i, (n, N, M, 1), iters=9) for i in range(2)]
        data = [build(w) for w in ws]
        plan = ct.Plan(n, N, M)
        args = ([gpu(d[1]) for d in data], 0.005, [ct.pack_mask(d[2]) for d in data],
                [gpu(d[3]) for d in data])
        made.append((plan, args))
    grouped = [ct.SolverBatch(p, *a, launch=NO_TUNE) for p, a in made]
    alone = [ct.SolverBatch(p, *a, launch=NO_TUNE) for p, a in made]
    grp = ct.SolverGroup(grouped)
    grp.step(9)
    for sv in alone:
        sv.step(9)
    for a, b in zip(grouped, alone):
        for x, y in zip(a.export(), b.export()):
            assert torch.equal(x, y)
    grouped[0].step(1)
    with pytest.raises(ct.CtpdError):
        grp.step(1)          # the group's solvers are no longer in step
    grp.close()


def test_batch_of_eight_512_equals_single():
    """Eight 512^2 x 720 x 768 problems in one batch solver, where the
    preconditioner's passes hold four row pairs (and four columns) per
    workgroup instead of one: each problem's state after two steps is
    bitwise that of a single solver with the batch's launch choices."""
    print("batch of eight at 512", flush=True)
    n, N, M = 512, 720, 768
    rng = np.random.default_rng(8)
    plan = ct.Plan(n, N, M)
    sinos = [gpu(50.0 * np.abs(rng.standard_normal((N, M)))) for _ in range(8)]
    sb = ct.SolverBatch(plan, sinos, 0.005, beta=600.0, c=2.0, launch=NO_TUNE)
    sb.step(2)
    ub, vb1b, vb2b = sb.export()
    lay, tvb = sb.layout(), sb.tuning()["tv_blocks"]
    launch = ct.Launch(tune=False, bp_slices=lay["bp_slices"], bp_kernel=lay["bp_kernel"],
                       tv_blocks=tvb or None, fuse_tv=tvb > 0, fwd_walk=lay["angles_per_walk"])
    for b in range(8):
        sv = ct.Solver(plan, sinos[b], 0.005, beta=600.0, c=2.0, launch=launch)
        sv.step(2)
        for x, y in zip(sv.export(), (ub[b], vb1b[b], vb2b[b])):
            assert torch.equal(x, y)
