"""GPU (HIP, gfx950) vs FP64 oracle parity, through the C ABI.

Inputs are drawn once (seeded), rounded to FP32 and handed to both sides; the
oracle computes in FP64 on the same FP32 values.  Tolerances (relative L2):
1e-5 for R_h, R_h^*, M^{-1} and one PDRQS1 step (the spec per-step
bound), 1e-6 for the pointwise kernels (a few FP32 roundings per element),
1e-4 for the image after a fixed number of iterations.
"""
import math
import os

import numpy as np
import pytest
import torch

import synth
from oracle import gap as ogap
from oracle import geometry, pdrq, power, precond, prox, radon, tv

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


# n, N, M, h, ds -- several tiles and a ragged tail, odd M, N = 1, detector
# narrower than the image diagonal, ds < h (strips without a pixel), h != 1
GEOMS = [
    (64, 90, 96, 1.0, 1.0),
    (54, 37, 81, 1.0, 1.0),
    (48, 61, 50, 1.0, 1.3),
    (40, 33, 64, 1.0, 0.8),
    (96, 1, 140, 1.0, 1.0),
    (2, 3, 4, 1.0, 1.0),
    (128, 180, 192, 0.7, 0.7),
    (100, 45, 150, 1.0, 1.0),
    (90, 180, 128, 1.0, 0.8),   # angle pairs, strips that can miss a row
    (90, 180, 128, 1.0, 1.4),   # pairs too wide for the paired kernel
    (66, 4, 100, 1.0, 1.0),     # one pair and two angles alone
    (63, 90, 96, 1.0, 1.0),     # odd n: the mirror pairs' centre column
    (65, 36, 100, 1.0, 1.0),    # odd n, a ragged left-half tile
    (33, 7, 50, 1.0, 1.0),      # odd N
]


def _plan_or_skip(n, N, M, h=1.0, ds=1.0, bp_kernel="auto"):
    """A plan with the given backprojector; the pair kernels need angles that
    pair as theta, pi - theta (CT_E_UNSUPPORTED otherwise: skipped)."""
    try:
        return ct.Plan(n, N, M, h, ds, bp_kernel=bp_kernel)
    except ct.CtpdError as e:
        if bp_kernel != "auto" and e.code == -2:
            pytest.skip("angles do not pair")
        raise


@pytest.mark.parametrize("kern", ["auto", "pairs8"])
@pytest.mark.parametrize("geo", GEOMS, ids=lambda g: "x".join(map(str, g)))
def test_radon_pair_parity(geo, kern):
    """R_h and R_h^* against the oracle on each geometry, with the plan's
    default backprojector and with the mirror pairs on 32 x 64 tiles (8
    pixels per thread; one 64-bin staging round per segment where ds/h is
    large enough)."""
    n, N, M, h, ds = geo
    print("radon parity", geo, kern, flush=True)
    g = geometry.Geometry(n, N, M, h, ds)
    rng = np.random.default_rng(n * 1000 + N)
    x = f32(rng.uniform(-1, 1, (n, n)))
    y = f32(rng.uniform(-1, 1, (N, M)))
    plan = _plan_or_skip(n, N, M, h, ds, kern)
    fx = host(plan.radon_fwd(gpu(x)))
    by = host(plan.radon_adj(gpu(y)))
    assert rel(fx, radon.radon_fwd(g, x)) <= 1e-5
    assert rel(by, radon.radon_adj(g, y)) <= 1e-5
    # the GPU pair is adjoint to FP32 summation accuracy
    lhs, rhs = np.sum(fx * y), np.sum(x * by)
    assert abs(lhs - rhs) <= 2e-6 * np.linalg.norm(fx) * np.linalg.norm(y)


WALK_GEOMS = [(64, 90, 96, 1.0, 1.0), (63, 92, 96, 1.0, 1.0), (128, 180, 192, 0.7, 0.7),
              (96, 1, 140, 1.0, 1.0), (66, 6, 100, 1.0, 1.0), (90, 180, 128, 1.0, 1.4),
              (90, 180, 128, 1.0, 0.8)]


@pytest.mark.parametrize("walk", [1, 2, 4])
@pytest.mark.parametrize("geo", WALK_GEOMS, ids=lambda g: "x".join(map(str, g)))
def test_forward_projector_walk_modes(geo, walk):
    """R_h with one, two or four angles per walk (theta, pi/2 - theta,
    pi - theta, pi/2 + theta; a mode whose windows do not fit, or whose angles
    do not group, falls back to the next) against the oracle, on geometries
    with incomplete quadruples (N = 92, 6, 1), ds != h and odd n; the mode the
    plan took is at most the one asked for."""
    n, N, M, h, ds = geo
    print("walk modes", geo, walk, flush=True)
    g = geometry.Geometry(n, N, M, h, ds)
    rng = np.random.default_rng(n * 7 + N)
    x = f32(rng.uniform(-1, 1, (n, n)))
    plan = ct.Plan(n, N, M, h, ds, fwd_angles_per_walk=walk)
    fx = host(plan.radon_fwd(gpu(x)))
    assert rel(fx, radon.radon_fwd(g, x)) <= 1e-5
    assert plan.layout()["angles_per_walk"] <= walk


def test_pd_step_parity_four_angles_per_walk():
    """Two PDRQS1 steps with R_h walking four angles at a time (metal trace,
    tuned launch) against the oracle."""
    n, N, M = 128, 180, 192
    w, g, u0, mask, bound = _small_metal_problem(n, N, M)
    s = pdrq.setup(pdrq.Problem(g, u0, mask, bound, w.alpha), pdrq.Params(),
                   f32(w.start_norm), f32(w.start_precond))
    plan = ct.Plan(n, N, M, fwd_angles_per_walk=4)
    sv = ct.Solver(plan, gpu(u0), w.alpha, ct.pack_mask(mask), gpu(bound), beta=s.beta, c=s.c)
    assert sv.layout()["angles_per_walk"] == 4
    rng = np.random.default_rng(12)
    u = f32(0.02 * rng.uniform(0, 1, (n, n)))
    vb1 = f32(0.01 * rng.standard_normal((N, M)))
    vb2 = f32(s.lam_t / s.params.tau * rng.standard_normal((2, n, n)))
    sv.import_state(gpu(u), gpu(vb1), gpu(vb2))
    sv.step(2)
    gu, g1, g2 = (host(t) for t in sv.export())
    st = pdrq.step(s, pdrq.step(s, pdrq.state_from(s, u, vb1, vb2)))
    assert rel(gu, st.u) <= 2e-5
    assert rel(g1, st.vb1) <= 2e-5
    assert rel(g2, st.vb2) <= 1e-4


@pytest.mark.parametrize("walk", [1, 2, 4])
def test_pd_step_parity_solver_walk(walk):
    """A solver whose iteration walks 1, 2 or 4 angles at a time on a plan
    whose own walk is 2 (its standalone calls keep it): two PDRQS1 steps
    against the oracle."""
    n, N, M = 128, 180, 192
    print("solver walk", walk, flush=True)
    w, g, u0, mask, bound = _small_metal_problem(n, N, M)
    s = pdrq.setup(pdrq.Problem(g, u0, mask, bound, w.alpha), pdrq.Params(),
                   f32(w.start_norm), f32(w.start_precond))
    plan = ct.Plan(n, N, M)
    assert plan.layout()["angles_per_walk"] == 2
    sv = ct.Solver(plan, gpu(u0), w.alpha, ct.pack_mask(mask), gpu(bound), beta=s.beta, c=s.c,
                   launch=ct.Launch(fwd_walk=walk))
    assert sv.layout()["angles_per_walk"] == walk
    assert plan.layout()["angles_per_walk"] == 2
    rng = np.random.default_rng(12)
    u = f32(0.02 * rng.uniform(0, 1, (n, n)))
    vb1 = f32(0.01 * rng.standard_normal((N, M)))
    vb2 = f32(s.lam_t / s.params.tau * rng.standard_normal((2, n, n)))
    sv.import_state(gpu(u), gpu(vb1), gpu(vb2))
    sv.step(2)
    gu, g1, g2 = (host(t) for t in sv.export())
    st = pdrq.step(s, pdrq.step(s, pdrq.state_from(s, u, vb1, vb2)))
    assert rel(gu, st.u) <= 2e-5
    assert rel(g1, st.vb1) <= 2e-5
    assert rel(g2, st.vb2) <= 1e-4


def test_tuning_times_the_walks():
    """The set-up tuning times R_h with each number of angles per walk the
    angles allow (4, 2 and 1 here), keeps a walk fixed by the plan, and
    rejects an unknown walk."""
    n, N, M = 128, 180, 192
    w, g, u0, mask, bound = _small_metal_problem(n, N, M)
    args = (gpu(u0), w.alpha, ct.pack_mask(mask), gpu(bound))
    tuned = ct.Solver(ct.Plan(n, N, M), *args, beta=500.0, c=2.0)
    t = tuned.tuning()
    assert t["source"] == "timed"
    # 3 walks, at least 2 backprojector choices and 2 update placements
    assert t["timed"] >= 3 + 2 + 2
    assert tuned.layout()["angles_per_walk"] in (1, 2, 4)
    one = ct.Solver(ct.Plan(n, N, M, fwd_angles_per_walk=1), *args, beta=500.0, c=2.0)
    assert one.layout()["angles_per_walk"] == 1
    with pytest.raises(ct.CtpdError):
        ct.Solver(ct.Plan(n, N, M), *args, beta=500.0, c=2.0, launch=ct.Launch(fwd_walk=3))


@pytest.mark.parametrize("geo", [(64, 90, 96), (63, 90, 96), (2, 3, 4), (100, 60, 150)],
                         ids=lambda g: "x".join(map(str, g)))
def test_backprojection_with_and_without_mirror_pairs(geo):
    """The mirror-pair backprojector (theta and pi - theta from one bin
    coordinate; 4 or 8 pixels per thread) and the one-angle backprojector
    agree with the oracle and with each other to FP32 summation accuracy."""
    n, N, M = geo
    print("backprojection pairs", geo, flush=True)
    g = geometry.Geometry(n, N, M)
    rng = np.random.default_rng(n + N)
    y = f32(rng.uniform(-1, 1, (N, M)))
    ref = radon.radon_adj(g, y)
    out = {}
    for kern in ("one_angle", "pairs4", "pairs8"):
        plan = ct.Plan(n, N, M, bp_kernel=kern)
        out[kern] = host(plan.radon_adj(gpu(y)))
        assert rel(out[kern], ref) <= 1e-5
    assert rel(out["pairs4"], out["one_angle"]) <= 1e-6
    assert rel(out["pairs8"], out["one_angle"]) <= 1e-6


def test_radon_deterministic_and_arbitrary_angles():
    """Angles need not be uniform or sorted (§3.1 allows any theta_l); results
    are bitwise reproducible (no atomics)."""
    n, N, M = 64, 50, 96
    rng = np.random.default_rng(7)
    ang = rng.uniform(0, 2 * math.pi, N)
    plan = ct.Plan(n, N, M, angles=ang)
    g = geometry.Geometry(n, N, M, thetas=tuple(ang))
    x = f32(rng.uniform(0, 1, (n, n)))
    y = f32(rng.uniform(-1, 1, (N, M)))
    a = host(plan.radon_fwd(gpu(x)))
    b = host(plan.radon_fwd(gpu(x)))
    assert np.array_equal(a, b)
    assert rel(a, radon.radon_fwd(g, x)) <= 1e-5
    c = host(plan.radon_adj(gpu(y)))
    assert np.array_equal(c, host(plan.radon_adj(gpu(y))))
    assert rel(c, radon.radon_adj(g, y)) <= 1e-5


def test_grad_div_prox_parity():
    rng = np.random.default_rng(3)
    for n, h in ((64, 1.0), (45, 0.5)):
        u = f32(rng.standard_normal((n, n)))
        p = f32(rng.standard_normal((2, n, n)))
        assert rel(host(ct.grad(gpu(u), h)), tv.grad(u, h)) <= 1e-6
        assert rel(host(ct.div(gpu(p), h)), tv.div(p, h)) <= 1e-6
        q = f32(rng.standard_normal((2, n, n)))
        for r in (0.0, 0.3, 10.0):
            assert rel(host(ct.tv_project(gpu(q), r)) + 1e-30, prox.tv_project(q, r) + 1e-30) <= 1e-6
    N, M = 37, 70
    q = f32(rng.standard_normal((N, M)))
    u0 = f32(rng.standard_normal((N, M)))
    bd = f32(rng.standard_normal((N, M)))
    mask = rng.uniform(size=(N, M)) < 0.3
    for s in (0.5, 1.0, 2.0):
        got = host(ct.prox_sino(gpu(q), s, gpu(u0), gpu(bd), ct.pack_mask(mask)))
        assert rel(got, prox.prox_sino(q, s, u0, bd, mask)) <= 1e-6
        got = host(ct.prox_sino(gpu(q), s, gpu(u0), None, None))
        assert rel(got, prox.prox_sino(q, s, u0, bd, np.zeros_like(mask))) <= 1e-6


@pytest.mark.parametrize("n", [2, 6, 8, 32, 48, 64, 96, 128, 162, 256, 384, 512, 768, 1024, 2048, 4096])
def test_precond_parity(n):
    print("precond parity", n, flush=True)
    rng = np.random.default_rng(n)
    y = f32(rng.standard_normal((n, n)))
    sig, tau, c, eps = 1.0, 1 / math.sqrt(8), 0.7, 0.3
    pc = ct.Precond(n, sig, tau, c, eps)
    got = host(pc.apply(gpu(y)))
    assert rel(got, precond.precond_inverse(y, sig, tau, c, eps)) <= 1e-5


def test_power_norm_parity():
    w = synth.workload("C1")
    g = geometry.Geometry(w.n, w.n_angles, w.n_bins)
    x0 = f32(w.start_norm)
    plan = ct.Plan(w.n, w.n_angles, w.n_bins)
    b_gpu = ct.power_norm(plan, 30, gpu(x0))
    b_ref = power.radon_norm(lambda u: radon.radon_fwd(g, u), lambda v: radon.radon_adj(g, v), x0, 30)
    assert abs(b_gpu - b_ref) <= 1e-5 * b_ref


def _small_metal_problem(n=64, N=90, M=96):
    w = synth.workload("C2", n=n, n_angles=N, n_bins=M)
    g, u0, mask, bound = build(w)
    return w, g, u0, mask, bound


def test_setup_constants_parity():
    """beta (||R_h||) and c from the GPU's FP32 operators with FP64 norms match
    the FP64 oracle's power iterations from the same start images."""
    w, g, u0, mask, bound = _small_metal_problem()
    plan = ct.Plan(g.n, g.n_angles, g.n_bins)
    sv = ct.Solver(plan, gpu(u0), w.alpha, ct.pack_mask(mask), gpu(bound),
                   start_norm=gpu(f32(w.start_norm)), start_precond=gpu(f32(w.start_precond)))
    info = sv.info()
    s = pdrq.setup(pdrq.Problem(g, u0, mask, bound, w.alpha), pdrq.Params(),
                   f32(w.start_norm), f32(w.start_precond))
    assert abs(info["beta"] - s.beta) <= 1e-5 * s.beta
    assert abs(info["c"] - s.c) <= 1e-5 * s.c
    assert abs(info["lam_t"] - s.lam_t) <= 1e-5 * s.lam_t


@pytest.mark.parametrize("size", [(64, 90, 96), (54, 41, 80)])
def test_pd_step_parity(size):
    """One PDRQS1 step from the same (random) state, with the same beta and c."""
    n, N, M = size
    w, g, u0, mask, bound = _small_metal_problem(n, N, M)
    s = pdrq.setup(pdrq.Problem(g, u0, mask, bound, w.alpha), pdrq.Params(),
                   f32(w.start_norm), f32(w.start_precond))
    plan = ct.Plan(n, N, M)
    sv = ct.Solver(plan, gpu(u0), w.alpha, ct.pack_mask(mask), gpu(bound), beta=s.beta, c=s.c)
    rng = np.random.default_rng(11)
    u = f32(rng.uniform(0, 1, (n, n)))
    vb1 = f32(0.01 * rng.standard_normal((N, M)))
    vb2 = f32(s.lam_t / s.params.tau * rng.standard_normal((2, n, n)))
    sv.import_state(gpu(u), gpu(vb1), gpu(vb2))
    sv.step(1)
    gu, g1, g2 = (host(t) for t in sv.export())
    st = pdrq.step(s, pdrq.state_from(s, u, vb1, vb2))
    assert rel(gu, st.u) <= 1e-5
    assert rel(g1, st.vb1) <= 1e-5
    assert rel(g2, st.vb2) <= 1e-5
    # a second step continues from the GPU-kept caches
    sv.step(1)
    gu2 = host(sv.export()[0])
    st2 = pdrq.step(s, st)
    assert rel(gu2, st2.u) <= 2e-5


@pytest.mark.parametrize("slices,kern", [(1, "pairs4"), (3, "pairs4"), (16, "pairs4"),
                                         (16, "one_angle"), (5, "one_angle"), (12, "pairs4"),
                                         (4, "pairs8"), (16, "pairs8"), (12, "pairs8")])
def test_pd_step_parity_slices_and_backprojectors(slices, kern):
    """Two PDRQS1 steps with a fixed number of angle slices (their sum and
    epilogue formed in the FFT row pass, or by the combine pass for a count it
    does not take) and each backprojector, against the oracle."""
    n, N, M = 64, 90, 96
    print("pd step slices", slices, kern, flush=True)
    w, g, u0, mask, bound = _small_metal_problem(n, N, M)
    s = pdrq.setup(pdrq.Problem(g, u0, mask, bound, w.alpha), pdrq.Params(),
                   f32(w.start_norm), f32(w.start_precond))
    plan = ct.Plan(n, N, M)
    sv = ct.Solver(plan, gpu(u0), w.alpha, ct.pack_mask(mask), gpu(bound), beta=s.beta, c=s.c,
                   launch=ct.Launch(bp_slices=slices, bp_kernel=kern))
    lay = sv.layout()
    assert lay["bp_slices"] == slices
    assert lay["bp_angles_per_position"] == (1 if kern == "one_angle" else 2)
    assert lay["bp_pair_pixels"] == {"one_angle": 0, "pairs4": 4, "pairs8": 8}[kern]
    rng = np.random.default_rng(12)
    u = f32(rng.uniform(0, 1, (n, n)))
    vb1 = f32(0.01 * rng.standard_normal((N, M)))
    vb2 = f32(s.lam_t / s.params.tau * rng.standard_normal((2, n, n)))
    sv.import_state(gpu(u), gpu(vb1), gpu(vb2))
    sv.step(2)
    gu, g1, g2 = (host(t) for t in sv.export())
    st = pdrq.step(s, pdrq.step(s, pdrq.state_from(s, u, vb1, vb2)))
    assert rel(gu, st.u) <= 2e-5
    assert rel(g1, st.vb1) <= 2e-5
    assert rel(g2, st.vb2) <= 2e-5


def test_tuning_is_cached_per_plan_and_batch_size():
    """A second solver of the same batch size on a plan reuses the first
    one's tuned choice without timing; a batch of another size is timed on
    its own; each solver keeps its own choice (solvers created later change
    neither its layout nor its results); all match the oracle's step."""
    n, N, M = 64, 90, 96
    print("tuning cache", flush=True)
    w, g, u0, mask, bound = _small_metal_problem(n, N, M)
    s = pdrq.setup(pdrq.Problem(g, u0, mask, bound, w.alpha), pdrq.Params(),
                   f32(w.start_norm), f32(w.start_precond))
    plan = ct.Plan(n, N, M)
    args = (gpu(u0), w.alpha, ct.pack_mask(mask), gpu(bound))
    first = ct.Solver(plan, *args, beta=s.beta, c=s.c)
    t0 = first.tuning()
    assert t0["source"] == "timed" and t0["timed"] > 1
    lay0 = first.layout()
    first.step(1)
    ref1 = host(first.export()[0])
    second = ct.Solver(plan, *args, beta=s.beta, c=s.c)
    assert second.tuning()["source"] == "plan" and second.tuning()["timed"] == 0
    assert second.layout() == lay0
    batch = ct.SolverBatch(plan, [args[0], args[0]], w.alpha, [args[2], args[2]],
                           [args[3], args[3]], beta=s.beta, c=s.c)
    assert batch.tuning()["source"] == "timed"
    # a solver whose choice is fixed otherwise, created after the first one
    other = "one_angle" if lay0["bp_pair_pixels"] else "pairs4"
    other_walk = 1 if lay0["angles_per_walk"] != 1 else 2
    fixed = ct.Solver(plan, *args, beta=s.beta, c=s.c,
                      launch=ct.Launch(bp_kernel=other, bp_slices=3, tv_blocks=64,
                                       fwd_walk=other_walk))
    assert fixed.tuning()["source"] == "fixed"
    assert fixed.layout()["angles_per_walk"] == other_walk
    assert first.layout() == lay0
    st = pdrq.step(s, pdrq.zero_state(s))
    assert rel(ref1, st.u) <= 1e-5
    # the first solver's kernels are unchanged: from the zero state again,
    # its first iterate is bitwise the same
    first.import_state(*(gpu(a) for a in (np.zeros((n, n)), np.zeros((N, M)),
                                          np.zeros((2, n, n)))))
    first.step(1)
    assert np.array_equal(host(first.export()[0]), ref1)
    for sv in (second, fixed):
        sv.step(1)
        assert rel(host(sv.export()[0]), st.u) <= 1e-5


def test_tune_cache_file(tmp_path):
    """The tuning result goes to the JSON file named by the params; a solver
    on a new plan of the same geometry reads it instead of timing, and its
    iterates are bitwise those of the first solver (same kernels, same slice
    count, so the same FP32 summation order)."""
    import json
    n, N, M = 64, 90, 96
    path = str(tmp_path / "tune.json")
    w, g, u0, mask, bound = _small_metal_problem(n, N, M)
    args = (gpu(u0), w.alpha, ct.pack_mask(mask), gpu(bound))
    a = ct.Solver(ct.Plan(n, N, M), *args, beta=500.0, c=2.0,
                  launch=ct.Launch(tune_cache=path))
    assert a.tuning()["source"] == "timed" and a.tuning()["saved"]
    doc = json.load(open(path))
    assert len(doc["entries"]) == 1
    assert doc["entries"][0]["fwd_walk"] == a.layout()["angles_per_walk"]
    b = ct.Solver(ct.Plan(n, N, M), *args, beta=500.0, c=2.0,
                  launch=ct.Launch(tune_cache=path))
    assert b.tuning()["source"] == "file" and b.tuning()["timed"] == 0
    assert b.layout() == a.layout()
    assert b.tuning()["tv_blocks"] == a.tuning()["tv_blocks"]
    a.step(7)
    b.step(7)
    for x, y in zip(a.export(), b.export()):
        assert torch.equal(x, y)
    # an entry without every field (a file of an older format) is not used:
    # the next solver times its choices and writes a whole entry back
    text = open(path).read()
    open(path, "w").write(text.replace(', "fwd_walk": %d' % doc["entries"][0]["fwd_walk"], ""))
    assert "fwd_walk" not in open(path).read()
    c = ct.Solver(ct.Plan(n, N, M), *args, beta=500.0, c=2.0,
                  launch=ct.Launch(tune_cache=path))
    assert c.tuning()["source"] == "timed" and c.tuning()["saved"]
    assert json.load(open(path))["entries"][0]["fwd_walk"] == c.layout()["angles_per_walk"]


_CHILD = r"""
import sys
import numpy as np
import torch
import paper_1810_03275_amd as ct
z = np.load(sys.argv[1])
dev = torch.device("cuda")
t = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(dev)
n, N, M = (int(v) for v in z["shape"])
sv = ct.Solver(ct.Plan(n, N, M), t(z["u0"]), float(z["alpha"]), ct.pack_mask(z["mask"]), t(z["bound"]),
               beta=500.0, c=2.0, launch=ct.Launch(tune_cache=sys.argv[2]))
assert sv.tuning()["source"] == "file", sv.tuning()
sv.step(7)
np.savez(sys.argv[3], *[x.cpu().numpy() for x in sv.export()])
"""


def test_tune_cache_second_process(tmp_path):
    """A second process that reads the tuning file makes the same launch
    choices without timing and gives bitwise the same iterates as the
    process that wrote it."""
    import subprocess
    import sys
    n, N, M = 64, 90, 96
    path = str(tmp_path / "tune.json")
    w, g, u0, mask, bound = _small_metal_problem(n, N, M)
    a = ct.Solver(ct.Plan(n, N, M), gpu(u0), w.alpha, ct.pack_mask(mask), gpu(bound), beta=500.0,
                  c=2.0, launch=ct.Launch(tune_cache=path))
    assert a.tuning()["source"] == "timed" and a.tuning()["saved"]
    a.step(7)
    mine = [x.cpu().numpy() for x in a.export()]
    inp, out = str(tmp_path / "in.npz"), str(tmp_path / "out.npz")
    np.savez(inp, shape=np.array([n, N, M]), u0=u0, alpha=w.alpha, mask=mask, bound=bound)
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, "-c", _CHILD, inp, path, out], cwd=root,
                       capture_output=True, text=True, timeout=240)
    assert r.returncode == 0, r.stderr[-2000:]
    z = np.load(out)
    for k, x in enumerate(mine):
        assert np.array_equal(z[f"arr_{k}"], x)


@pytest.mark.parametrize("hook", ["fuse_tv", "defer", "tv_blocks"])
def test_fusions_are_bitwise_neutral(hook):
    """The gradient-side update run inside R_h's launch (with any number of
    extra workgroups), and the slice sum formed in the FFT row pass, do the
    same arithmetic in the same order as the separate kernels: the states
    after a few iterations are bitwise equal."""
    n, N, M = 64, 90, 96
    print("fusion neutral", hook, flush=True)
    w, g, u0, mask, bound = _small_metal_problem(n, N, M)
    s = pdrq.setup(pdrq.Problem(g, u0, mask, bound, w.alpha), pdrq.Params(),
                   f32(w.start_norm), f32(w.start_precond))
    plan = ct.Plan(n, N, M)
    out = []
    variants = ({"tv_blocks": 7}, {"tv_blocks": 64}) if hook == "tv_blocks" else \
        ({hook: False}, {hook: True})
    for var in variants:
        la = ct.Launch(bp_slices=4, bp_kernel="pairs4", tv_blocks=var.get("tv_blocks", 64),
                       **{k: v for k, v in var.items() if k != "tv_blocks"})
        sv = ct.Solver(plan, gpu(u0), w.alpha, ct.pack_mask(mask), gpu(bound), beta=s.beta, c=s.c,
                       launch=la)
        sv.step(6)
        out.append([host(t) for t in sv.export()])
    for a, b in zip(*out):
        assert np.all(np.isfinite(a)) and np.array_equal(a, b)


def test_end_to_end_c1():
    """C1 (64^2, 90 x 96, alpha = 0.01, 200 iterations, no metal): the final
    image matches the oracle to 1e-4; the gap records agree."""
    w = synth.workload("C1")
    g, u0, mask, bound = build(w)
    assert not mask.any()
    plan = ct.Plan(g.n, g.n_angles, g.n_bins)
    u_gpu, rep = ct.reconstruct(plan, gpu(u0), w.alpha, None, None, k_max=w.iters, gap_every=50,
                                start_norm=gpu(f32(w.start_norm)),
                                start_precond=gpu(f32(w.start_precond)))
    s = pdrq.setup(pdrq.Problem(g, u0, mask, bound, w.alpha), pdrq.Params(),
                   f32(w.start_norm), f32(w.start_precond))
    st, recs = pdrq.run(s, w.iters, record_every=50)
    assert rel(host(u_gpu), st.u) <= 1e-4
    recs = np.array(recs)
    assert rep.shape == recs.shape
    assert np.allclose(rep[:, 0], recs[:, 0], rtol=1e-4)          # P
    assert np.allclose(rep[:, 1], recs[:, 1], rtol=1e-4)          # G*
    assert np.all(np.abs(rep[:, 2] - recs[:, 2]) <= 1e-4 * np.abs(recs[:, 0]))
    assert np.allclose(rep[:, 3], recs[:, 3], rtol=2e-2, atol=1e-6)
    assert np.allclose(rep[:, 5], recs[:, 5], rtol=2e-2, atol=1e-7)


def test_end_to_end_metal_small():
    """C2 recipe on a 64^2 slice (2 scaled metal discs, inequality constraints
    active on the metal trace): 100 iterations match the oracle to 1e-4."""
    w, g, u0, mask, bound = _small_metal_problem()
    assert mask.any()
    plan = ct.Plan(g.n, g.n_angles, g.n_bins)
    u_gpu, rep = ct.reconstruct(plan, gpu(u0), w.alpha, ct.pack_mask(mask), gpu(bound),
                                k_max=100, gap_every=100, start_norm=gpu(f32(w.start_norm)),
                                start_precond=gpu(f32(w.start_precond)))
    s = pdrq.setup(pdrq.Problem(g, u0, mask, bound, w.alpha), pdrq.Params(),
                   f32(w.start_norm), f32(w.start_precond))
    st, recs = pdrq.run(s, 100, record_every=100)
    assert rel(host(u_gpu), st.u) <= 1e-4
    assert rep[0, 4] == pytest.approx(recs[0][4], rel=1e-2, abs=1e-6)   # violation


def test_full_size_c2_sampled():
    """512^2, 720 x 768 in the benchmark's launch configuration: R_h and R_h^*
    spot-checked against the oracle at sampled outputs, and adjointness."""
    n, N, M = 512, 720, 768
    g = geometry.Geometry(n, N, M)
    rng = np.random.default_rng(5)
    x = f32(rng.uniform(0, 1, (n, n)))
    y = f32(rng.uniform(-1, 1, (N, M)))
    plan = ct.Plan(n, N, M)
    fx = host(plan.radon_fwd(gpu(x)))
    by = host(plan.radon_adj(gpu(y)))
    pix = [(int(j), int(i)) for j, i in rng.integers(0, n, (24, 2))] + [(0, 0), (n - 1, n - 1), (0, n - 1)]
    ref = radon.radon_adj_at(g, y, pix)
    got = np.array([by[j, i] for j, i in pix])
    assert rel(got, ref) <= 1e-5
    bins = [(int(l), int(k)) for l, k in zip(rng.integers(0, N, 40), rng.integers(100, 668, 40))]
    bins += [(0, 0), (N - 1, M - 1), (N // 4, M // 2), (N // 2, 30)]
    ref = radon.radon_fwd_at(g, x, bins)
    got = np.array([fx[l, k] for l, k in bins])
    assert rel(got, ref) <= 1e-5
    lhs, rhs = np.sum(fx * y), np.sum(x * by)
    assert abs(lhs - rhs) <= 2e-6 * np.linalg.norm(fx) * np.linalg.norm(y)
    # mass conservation per angle (every pixel projects inside: 512 sqrt 2 < 768)
    assert np.allclose(fx.sum(axis=1), x.sum(), rtol=2e-6)


def test_errors_from_gpu_side():
    plan = ct.Plan(64, 10, 96)
    with pytest.raises(ValueError):
        plan.radon_fwd(torch.zeros((64, 64)))            # CPU tensor: no CPU path
    with pytest.raises(ValueError):
        plan.radon_fwd(torch.zeros((63, 64), device=DEV))
    with pytest.raises(ct.CtpdError):
        ct.Solver(ct.Plan(50, 10, 80), torch.zeros((10, 80), device=DEV), 0.1)  # n = 50: not 2^a 3^b
    sv = ct.Solver(plan, torch.ones((10, 96), device=DEV), 0.1)
    with pytest.raises(ct.CtpdError):
        sv.gap()                                          # no iteration yet
    bad = torch.ones((10, 96), device=DEV)
    bad[3, 4] = float("nan")
    with pytest.raises(ct.CtpdError) as e:
        ct.Solver(plan, bad, 0.1, validate=True)
    assert e.value.code == -4


@pytest.mark.parametrize("walk", [None, 4, 1])
def test_graph_replay_matches_eager(walk):
    """k iterations replayed from the captured HIP graph give bitwise the same
    state as k single eager steps (same kernels, same order, no atomics), also
    when the solver's R_h walks another number of angles than the plan (its
    own forward tables, captured into the graph)."""
    print("graph replay, walk", walk, flush=True)
    w, g, u0, mask, bound = _small_metal_problem()
    plan = ct.Plan(g.n, g.n_angles, g.n_bins)
    kw = dict(beta=500.0, c=2.0, launch=ct.Launch(fwd_walk=walk))
    a = ct.Solver(plan, gpu(u0), w.alpha, ct.pack_mask(mask), gpu(bound), **kw)
    b = ct.Solver(plan, gpu(u0), w.alpha, ct.pack_mask(mask), gpu(bound), **kw)
    a.step(11)           # 5 graph replays of 2 iterations + 1 eager
    a.step(7)            # other parity: second graph
    a.step(37)           # 1 eager, 2 replays of 16 iterations, 2 of 2
    a.step(40)           # the other parity's long graph
    for _ in range(95):
        b.step(1)
    for x, y in zip(a.export(), b.export()):
        assert torch.equal(x, y)
    assert a.info()["iters"] == b.info()["iters"] == 95
    assert np.array_equal(a.gap(), b.gap())
    if walk is not None:
        assert a.layout()["angles_per_walk"] == walk
