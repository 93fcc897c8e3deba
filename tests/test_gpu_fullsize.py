"""Full-size parity of Algorithm PDRQS1 (§4.4) through the C ABI.

* 512^2 x 720 x 768 with 2 metal discs (the benchmark workload): one step
  from a seeded iterate against the oracle's step, element by element, and
  the FP64 record of that state (its metal-trace terms included); 500
  iterations from the zero state against the oracle's stored run
  (tests/golden/c2_pdrqs1_500.npz).
* 64^2 with metal: the record of one step from a shared state, every entry.
* 2048^2 x 2880 x 3072: one step from a seeded iterate on seeded problem data
  against the oracle's stored sampled entries (tests/golden/c5_step_sampled.npz),
  and 20 iterations from the zero state on the same kind of data
  (tests/golden/c5_pdrqs1_20_sampled.npz).
* The five image sizes of the uneven batch (256 ... 1024, N = 1.4 n,
  M = 1.5 n): one batched step per size against the oracle's stored sampled
  entries (tests/golden/c3_step_sampled.npz), and the batch bitwise equal to
  single solvers with the same launch choices.

Stored values are written by tests/golden/make_golden.py, which calls only
the oracle.  Tolerances (relative L2): 1e-5 per step (vb2: plus the error of
u_new carried through the gradient, vb2_tol) and for the record of a shared
state, 1e-4 for the image after 500 iterations.
"""
import os
import sys

import numpy as np
import pytest
import torch

import synth
from oracle import gap as ogap
from oracle import pdrq

from oracle_inputs import build, f32, random_problem, random_state

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))
import make_golden as mg  # noqa: E402

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


def golden(name):
    path = os.path.join(HERE, "golden", name)
    assert os.path.exists(path), f"missing stored oracle values {path}"
    return np.load(path)


def dual_scale(lam, beta):
    """lambda~/tau as the oracle's set-up forms it (the seeded vb2's scale)."""
    return (lam / beta ** 2) / pdrq.Params().tau


def vb2_tol(rel_u, norm_u, norm_vb2, h=1.0):
    """Tolerance (relative L2) of vb2 after one step.  vb2_new = vb2 + w - v2
    with v2 = vb2 + sigma tau grad u_new and w the projection of 2 v2 - vb2
    (§4.4): an error e of u_new reaches vb2 through sigma tau grad, whose norm
    is at most sigma tau sqrt(8) / h = 1 / h (sigma tau = 1 / sqrt 8), once in
    v2 and, through the nonexpansive projection, twice in w; so
    ||d vb2|| <= 3 ||e|| / h beyond vb2's own FP32 rounding (1e-5)."""
    return 1e-5 + 3.0 * rel_u * norm_u / (h * norm_vb2)


def check_step(got, new, h=1.0):
    """u and vb1 of a step to 1e-5, vb2 to vb2_tol."""
    ru, r1, r2 = (rel(a, b) for a, b in zip(got, (new.u, new.vb1, new.vb2)))
    assert ru <= 1e-5 and r1 <= 1e-5
    assert r2 <= vb2_tol(ru, np.linalg.norm(new.u), np.linalg.norm(new.vb2), h), (r2, ru)


def check_record(got, ref, tol):
    """The six record entries (P, G*, gap, rho_D, V, du) of a shared state.
    gap = P + G* is compared on the scale of |P| + |G*| (the two may nearly
    cancel); V is compared absolutely when the reference is zero."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    for q in (0, 1, 3, 5):
        assert abs(got[q] - ref[q]) <= tol * abs(ref[q]), (q, got[q], ref[q])
    assert abs(got[2] - ref[2]) <= tol * (abs(ref[0]) + abs(ref[1]))
    assert abs(got[4] - ref[4]) <= tol * max(abs(ref[4]), 1e-6 * abs(ref[0]) ** 0.5)


def one_step_vs_oracle(g, u0, mask, bound, lam, beta, c, seed, u_scale, launch=None):
    """GPU and oracle advance the same seeded iterate by one PDRQS1 step;
    returns (gpu state, oracle state, gpu record, oracle record, oracle setup,
    oracle y1)."""
    n, N, M = g.n, g.n_angles, g.n_bins
    s = pdrq.setup(pdrq.Problem(g, u0, mask, bound, lam), pdrq.Params(), beta=beta, c=c)
    u, vb1, vb2 = random_state(n, N, M, seed, s.lam_t / s.params.tau, u_scale)
    plan = ct.Plan(n, N, M)
    sv = ct.Solver(plan, gpu(u0), lam, ct.pack_mask(mask) if mask.any() else None,
                   gpu(bound) if mask.any() else None, beta=beta, c=c, launch=launch)
    sv.import_state(gpu(u), gpu(vb1), gpu(vb2))
    sv.step(1)
    got = [host(t) for t in sv.export()]
    rec_gpu = sv.gap()
    st = pdrq.state_from(s, u, vb1, vb2)
    new, y1, w = pdrq.step(s, st, return_dual=True)
    rec_ref = ogap.record(s, new.u, y1, w, u)
    return got, new, rec_gpu, rec_ref, s, y1


def test_gap_record_metal_small():
    """64^2 with two metal discs: from a shared seeded iterate, one step and
    the FP64 record on both sides; every entry agrees to 1e-5, and the
    record's metal-trace term (the sum over D0 of y1 C~ in G*) is a sizeable
    part of G* (so that the D0 branch of the record is exercised)."""
    w = synth.workload("C2", n=64, n_angles=90, n_bins=96)
    g, u0, mask, bound = build(w)
    assert mask.any()
    s0 = pdrq.setup(pdrq.Problem(g, u0, mask, bound, w.alpha), pdrq.Params(),
                    f32(w.start_norm), f32(w.start_precond))
    got, new, rec_gpu, rec_ref, s, y1 = one_step_vs_oracle(g, u0, mask, bound, w.alpha,
                                                           s0.beta, s0.c, 6401, mg.STEP_U_SCALE)
    print("metal small: rel u %.2e vb1 %.2e vb2 %.2e" % tuple(
        rel(a, b) for a, b in zip(got, (new.u, new.vb1, new.vb2))), flush=True)
    print("records", rec_gpu, rec_ref, flush=True)
    check_step(got, new, g.h)
    d0_term = float(np.sum((y1 * s.cb)[mask]))
    assert abs(d0_term) > 1e-3 * abs(rec_ref[1])
    check_record(rec_gpu, rec_ref, 1e-5)


def test_c2_one_step_and_record():
    """512^2 x 720 x 768 with 2 metal discs, the benchmark's launch
    configuration (tuned): one step from a seeded iterate matches the
    oracle's step in u and vb1 (1e-5) and vb2 (vb2_tol), and the FP64 records
    agree (1e-5)."""
    print("c2 one step", flush=True)
    w = synth.workload("C2")
    g, u0, mask, bound = build(w)
    got, new, rec_gpu, rec_ref, s, y1 = one_step_vs_oracle(g, u0, mask, bound, w.alpha,
                                                           600.0, 1.25, 5121, mg.STEP_U_SCALE)
    print("c2 one step: rel u %.2e vb1 %.2e vb2 %.2e" % tuple(
        rel(a, b) for a, b in zip(got, (new.u, new.vb1, new.vb2))), flush=True)
    print("records", rec_gpu, rec_ref, flush=True)
    d0_term = float(np.sum((y1 * s.cb)[mask]))
    assert abs(d0_term) > 1e-3 * abs(rec_ref[1])
    check_step(got, new, g.h)
    check_record(rec_gpu, rec_ref, 1e-5)


def test_c2_500_iterations():
    """The benchmark workload solved as the benchmark solves it (set-up by
    power iterations from the workload's start images, tuned launch, graph
    replay): beta and c match the oracle's (1e-5); after 500 iterations the
    image matches the oracle's stored run (1e-4), and the records after every
    100th iteration agree in P (1e-4), G* and the gap (to the first-order
    bound below: G* sums terms of both signs); rho_D, V and du are residuals
    of the iterate itself, so a 1e-5 difference of iterates makes them differ
    by more: 5e-2."""
    print("c2 500 iterations", flush=True)
    z = golden("c2_pdrqs1_500.npz")
    w = synth.workload("C2")
    g, u0, mask, bound = build(w)
    plan = ct.Plan(g.n, g.n_angles, g.n_bins)
    sv = ct.Solver(plan, gpu(u0), w.alpha, ct.pack_mask(mask), gpu(bound),
                   start_norm=gpu(f32(w.start_norm)), start_precond=gpu(f32(w.start_precond)))
    info = sv.info()
    assert abs(info["beta"] - float(z["beta"])) <= 1e-5 * float(z["beta"])
    assert abs(info["c"] - float(z["c"])) <= 1e-5 * float(z["c"])
    recs = []
    for _ in range(5):
        sv.step(100)
        recs.append(sv.gap())
    assert rel(host(sv.export()[0]), z["u"]) <= 1e-4
    ref = z["records"]
    for r, q, (ny1, nwg, nu) in zip(recs, ref, z["record_scales"]):
        assert abs(r[0] - q[0]) <= 1e-4 * abs(q[0])
        # G* = sum y1 (y1/2 + b) + sum_D0 y1 C~ moves to first order by
        # <dy1, wg> <= ||dy1|| ||wg||: with the dual iterate held to the
        # image's 1e-4, ||dy1|| <= 1e-4 ||y1||
        tol_g = 1e-4 * ny1 * nwg
        print("record: dG* %.3e (bound %.3e)" % (abs(r[1] - q[1]), tol_g), flush=True)
        assert abs(r[1] - q[1]) <= tol_g
        assert abs(r[2] - q[2]) <= 1e-4 * abs(q[0]) + tol_g
        assert r[3] == pytest.approx(q[3], rel=5e-2)
        assert r[4] == pytest.approx(q[4], rel=5e-2, abs=1e-6 * abs(q[0]) ** 0.5)
        assert r[5] == pytest.approx(q[5], rel=5e-2)


def test_c5_one_step_sampled():
    """2048^2 x 2880 x 3072: one step from a seeded iterate on seeded problem
    data (the inputs the stored oracle step used), in the launch
    configuration the benchmark's largest workload uses; the new u, vb1 and
    vb2 at the stored sampled pixels and bins match (1e-5; vb2: vb2_tol), and
    so do the three arrays' norms."""
    print("c5 one step", flush=True)
    z = golden("c5_step_sampled.npz")
    n, N, M = 2048, 2880, 3072
    u0, mask, bound = random_problem(N, M, mg.C5_PROBLEM_SEED)
    beta, c, lam = float(z["beta"]), float(z["c"]), float(z["lam"])
    u, vb1, vb2 = random_state(n, N, M, mg.C5_STATE_SEED, dual_scale(lam, beta),
                               mg.STEP_U_SCALE)
    plan = ct.Plan(n, N, M)
    sv = ct.Solver(plan, gpu(u0), lam, ct.pack_mask(mask), gpu(bound), beta=beta, c=c)
    del u0, bound
    sv.import_state(gpu(u), gpu(vb1), gpu(vb2))
    del u, vb1, vb2
    sv.step(1)
    gu, g1, g2 = sv.export()
    pix, bins = z["pix"], z["bins"]
    pj, pi = torch.as_tensor(pix[:, 0], device=DEV), torch.as_tensor(pix[:, 1], device=DEV)
    bl, bk = torch.as_tensor(bins[:, 0], device=DEV), torch.as_tensor(bins[:, 1], device=DEV)
    ru = rel(host(gu[pj, pi]), z["u"])
    assert ru <= 1e-5
    assert rel(host(g1[bl, bk]), z["vb1"]) <= 1e-5
    tol2 = vb2_tol(ru, z["norms"][0], z["norms"][2])
    print("c5: rel u %.2e, vb2 tolerance %.2e" % (ru, tol2), flush=True)
    assert rel(host(g2[0][pj, pi]), z["vb2_0"]) <= tol2
    assert rel(host(g2[1][pj, pi]), z["vb2_1"]) <= tol2
    norms = [float(torch.linalg.vector_norm(t.double())) for t in (gu, g1, g2)]
    assert rel(norms[:2], z["norms"][:2]) <= 1e-5
    assert abs(norms[2] - z["norms"][2]) <= tol2 * z["norms"][2]


def test_c5_20_iterations_sampled():
    """2048^2 x 2880 x 3072 on seeded problem data (the one-step check's kind),
    beta and c fixed: 20 PDRQS1 iterations from the zero state as the solver
    runs them (tuned launch, graph replay); the image at the stored sampled
    pixels and its norm match the oracle's run (1e-4, the bound for the image
    after a fixed iteration count), and so do vb1 at the sampled bins and the
    norm of vb1; vb2's norm within 1e-3 (it carries the image's error through
    the gradient, see vb2_tol)."""
    print("c5 20 iterations", flush=True)
    z = golden("c5_pdrqs1_20_sampled.npz")
    n, N, M = 2048, 2880, 3072
    u0, mask, bound = random_problem(N, M, mg.C5_PROBLEM_SEED)
    plan = ct.Plan(n, N, M)
    sv = ct.Solver(plan, gpu(u0), float(z["lam"]), ct.pack_mask(mask), gpu(bound),
                   beta=float(z["beta"]), c=float(z["c"]))
    del u0, bound
    sv.step(int(z["iters"]))
    gu, g1, g2 = sv.export()
    pix, bins = z["pix"], z["bins"]
    pj, pi = torch.as_tensor(pix[:, 0], device=DEV), torch.as_tensor(pix[:, 1], device=DEV)
    bl, bk = torch.as_tensor(bins[:, 0], device=DEV), torch.as_tensor(bins[:, 1], device=DEV)
    ru, r1 = rel(host(gu[pj, pi]), z["u"]), rel(host(g1[bl, bk]), z["vb1"])
    norms = [float(torch.linalg.vector_norm(t.double())) for t in (gu, g1, g2)]
    print("c5 20 iterations: rel u %.2e vb1 %.2e norms %s vs %s" % (ru, r1, norms, z["norms"]),
          flush=True)
    assert ru <= 1e-4 and r1 <= 1e-4
    assert rel(norms[:2], z["norms"][:2]) <= 1e-4
    assert abs(norms[2] - z["norms"][2]) <= 1e-3 * z["norms"][2]


def _launch_of(sv):
    """The launch choices a solver ended up with, as fixed params."""
    lay, tun = sv.layout(), sv.tuning()
    kern = lay["bp_kernel"]
    tvb = tun["tv_blocks"]
    return ct.Launch(bp_slices=lay["bp_slices"], bp_kernel=kern, tv_blocks=tvb or None,
                     fuse_tv=tvb > 0, fwd_walk=lay["angles_per_walk"])


@pytest.mark.parametrize("n", mg.C3_SIZES)
def test_c3_shape_batched_step(n):
    """Each image size of the uneven batch: two problems (seeded data and
    iterates) advanced as one batch solver with tuned launch choices, one
    step; each problem's new state at the stored sampled pixels and bins
    matches the oracle (1e-5; vb2: vb2_tol), and single solvers with the batch's launch
    choices give bitwise the batch's state."""
    print("c3 shape", n, flush=True)
    z = golden("c3_step_sampled.npz")
    n, N, M = mg.c3_geometry(n)
    beta, c, lam = mg.c3_beta(n), mg.C3_C, mg.C3_LAMBDA
    probs, states = [], []
    for b in range(2):
        ps, ss, _ = mg.c3_seeds(n, b)
        probs.append(random_problem(N, M, ps))
        states.append(random_state(n, N, M, ss, dual_scale(lam, beta), mg.STEP_U_SCALE))
    plan = ct.Plan(n, N, M)
    sinos = [gpu(p[0]) for p in probs]
    masks = [ct.pack_mask(p[1]) for p in probs]
    bounds = [gpu(p[2]) for p in probs]
    sb = ct.SolverBatch(plan, sinos, lam, masks, bounds, beta=beta, c=c)
    stack = [torch.stack([gpu(states[b][q]) for b in range(2)]) for q in range(3)]
    sb.import_state(*stack)
    sb.step(1)
    bu, b1, b2 = sb.export()
    launch = _launch_of(sb)
    for b in range(2):
        pre = f"n{n}_b{b}_"
        pix, bins = z[pre + "pix"], z[pre + "bins"]
        pj, pi = torch.as_tensor(pix[:, 0], device=DEV), torch.as_tensor(pix[:, 1], device=DEV)
        bl, bk = torch.as_tensor(bins[:, 0], device=DEV), torch.as_tensor(bins[:, 1], device=DEV)
        ru = rel(host(bu[b][pj, pi]), z[pre + "u"])
        assert ru <= 1e-5
        assert rel(host(b1[b][bl, bk]), z[pre + "vb1"]) <= 1e-5
        tol2 = vb2_tol(ru, z[pre + "norms"][0], z[pre + "norms"][2])
        assert rel(host(b2[b][0][pj, pi]), z[pre + "vb2_0"]) <= tol2
        assert rel(host(b2[b][1][pj, pi]), z[pre + "vb2_1"]) <= tol2
        sv = ct.Solver(plan, sinos[b], lam, masks[b], bounds[b], beta=beta, c=c, launch=launch)
        sv.import_state(*(gpu(a) for a in states[b]))
        sv.step(1)
        for x, y in zip(sv.export(), (bu[b], b1[b], b2[b])):
            assert torch.equal(x, y)
