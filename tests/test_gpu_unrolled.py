"""Differentiation on the GPU: RadonFn (backward = R_h^*) and K unrolled
PDRQS1 iterations (reverse sweep with checkpoints) against the FP64 oracle's
reverse mode and against finite differences of the GPU map itself."""
import numpy as np
import pytest
import torch

import synth
from oracle import pdrq, radon, unrolled

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


def test_radonfn_backward_is_adjoint_and_fd():
    """autograd through RadonFn gives R_h^* of the incoming gradient; a
    quadratic loss's central difference matches it exactly up to FP32."""
    print("radonfn", flush=True)
    n, N, M = 40, 33, 60
    plan = ct.Plan(n, N, M)
    rng = np.random.default_rng(4)
    x = gpu(rng.uniform(-1, 1, (n, n))).requires_grad_(True)
    b = gpu(rng.uniform(-1, 1, (N, M)))
    loss = 0.5 * ((ct.RadonFn.apply(x, plan) - b) ** 2).sum()
    loss.backward()
    r = plan.radon_fwd(x.detach()) - b
    assert rel(host(x.grad), host(plan.radon_adj(r))) <= 1e-6
    d = gpu(rng.uniform(-1, 1, (n, n)))
    e = 1e-2
    with torch.no_grad():
        lp = 0.5 * ((plan.radon_fwd(x + e * d) - b) ** 2).double().sum()
        lm = 0.5 * ((plan.radon_fwd(x - e * d) - b) ** 2).double().sum()
    fd = float((lp - lm) / (2 * e))
    an = float((x.grad.double() * d.double()).sum())
    assert an == pytest.approx(fd, rel=2e-4)
    y = gpu(rng.uniform(-1, 1, (N, M))).requires_grad_(True)
    (ct.RadonAdjFn.apply(y, plan) * x.detach()).sum().backward()
    assert rel(host(y.grad), host(plan.radon_fwd(x.detach()))) <= 1e-6


def _problem(seed, n=32, N=45, M=48, metal=1):
    w = synth.batched_workload(seed, (n, N, M, metal), iters=12)
    g, u0, mask, bound = build(w)
    truth = f32(w.phantom)
    return w, g, u0, mask, bound, truth


@pytest.mark.parametrize("K,every", [(12, 5), (9, 10)])
def test_unrolled_gradients_match_oracle(K, every):
    """u_K, dL/du0 and dL/dlambda of an MSE loss after K iterations (ragged last
    segment, and a single segment) against the oracle's reverse mode with the
    same beta and c."""
    print("unrolled vs oracle", K, every, flush=True)
    w, g, u0, mask, bound, truth = _problem(3)
    assert mask.any()
    plan = ct.Plan(g.n, g.n_angles, g.n_bins)
    lam = 0.02
    sino = gpu(u0)[None].requires_grad_(True)
    lt = torch.tensor(lam, device=DEV, requires_grad=True)
    mb, bd = [ct.pack_mask(mask)], [gpu(bound)]
    u = ct.unrolled_pd(plan, sino, lt, mb, bd, K=K, every=every)
    L = ((u[0] - gpu(truth)) ** 2).mean()
    L.backward()
    # the oracle with the GPU's beta and c
    probe = ct.Solver(plan, gpu(u0), lam, mb[0], bd[0])
    inf = probe.info()
    s = pdrq.setup(pdrq.Problem(g, u0, mask, bound, lam), pdrq.Params(), beta=inf["beta"],
                   c=inf["c"])
    states = unrolled.forward(s, K)
    Lo, gbar = unrolled.mse_loss(states[-1].u, truth)
    du0, dlam = unrolled.backward(s, states, gbar)
    assert rel(host(u[0]), states[-1].u) <= 1e-5
    assert rel(host(sino.grad[0]), du0) <= 1e-4
    assert float(lt.grad) == pytest.approx(dlam, rel=1e-4)
    assert np.all(host(sino.grad[0])[mask] == 0.0)


def test_unrolled_batch_equals_single():
    """Two problems as one batch: each problem's gradients equal its own
    single-problem gradients; the lambda gradient of the batch is their sum."""
    print("unrolled batch", flush=True)
    items = [_problem(5 + i, metal=i) for i in range(2)]
    plan = ct.Plan(32, 45, 48)
    lam = 0.02
    K, every = 8, 3
    sinos = torch.stack([gpu(it[2]) for it in items]).requires_grad_(True)
    lt = torch.tensor(lam, device=DEV, requires_grad=True)
    masks = [ct.pack_mask(it[3]) for it in items]
    bounds = [gpu(it[4]) for it in items]
    truths = torch.stack([gpu(it[5]) for it in items])
    u = ct.unrolled_pd(plan, sinos, lt, masks, bounds, K=K, every=every)
    ((u - truths) ** 2).mean(dim=(1, 2)).sum().backward()
    total = 0.0
    for b in range(2):
        s1 = gpu(items[b][2])[None].requires_grad_(True)
        l1 = torch.tensor(lam, device=DEV, requires_grad=True)
        u1 = ct.unrolled_pd(plan, s1, l1, [masks[b]], [bounds[b]], K=K, every=every)
        ((u1[0] - truths[b]) ** 2).mean().backward()
        assert rel(host(u1[0]), host(u[b])) <= 1e-6
        assert rel(host(s1.grad[0]), host(sinos.grad[b])) <= 1e-5
        total += float(l1.grad)
    assert float(lt.grad) == pytest.approx(total, rel=1e-5)


def test_unrolled_lambda_fd_on_gpu():
    """Central difference of the GPU map itself in lambda (relative step 5e-2,
    large enough to rise above FP32 rounding of the forward map) agrees with
    the reverse sweep to 5 % (the oracle comparison above is the tight one)."""
    print("unrolled fd", flush=True)
    w, g, u0, mask, bound, truth = _problem(9, n=48, N=67, M=72, metal=0)
    plan = ct.Plan(g.n, g.n_angles, g.n_bins)
    lam, K = 0.05, 10
    sino = gpu(u0)[None]
    tr = gpu(truth)
    probe = ct.Solver(plan, sino[0], lam)
    opts = dict(beta=probe.info()["beta"], c=probe.info()["c"])

    def loss(lv, grad=False):
        lt = torch.tensor(lv, device=DEV, requires_grad=grad)
        u = ct.unrolled_pd(plan, sino, lt, K=K, every=4, **opts)
        L = ((u[0] - tr) ** 2).double().mean()
        if grad:
            L.backward()
            return float(L.detach()), float(lt.grad)
        return float(L)

    _, an = loss(lam, True)
    d = 5e-2 * lam
    fd = (loss(lam + d) - loss(lam - d)) / (2 * d)
    assert an == pytest.approx(fd, rel=5e-2)


@pytest.fixture(scope="module")
def oracle_128():
    """A 128^2 x 179 x 192 problem with metal (the uneven batch's shape rule
    N = 1.4 n, M = 1.5 n), the GPU's beta and c, and the oracle's reverse
    mode of 6 unrolled iterations (MSE loss against the phantom)."""
    w, g, u0, mask, bound, truth = _problem(11, n=128, N=179, M=192, metal=2)
    assert mask.any()
    plan = ct.Plan(g.n, g.n_angles, g.n_bins)
    lam = 0.02
    probe = ct.Solver(plan, gpu(u0), lam, ct.pack_mask(mask), gpu(bound))
    inf = probe.info()
    s = pdrq.setup(pdrq.Problem(g, u0, mask, bound, lam), pdrq.Params(), beta=inf["beta"],
                   c=inf["c"])
    K = 6
    states = unrolled.forward(s, K)
    _, gbar = unrolled.mse_loss(states[-1].u, truth)
    du0, dlam = unrolled.backward(s, states, gbar)
    return dict(plan=plan, u0=u0, mask=mask, bound=bound, truth=truth, lam=lam, K=K,
                beta=inf["beta"], c=inf["c"], uK=states[-1].u, du0=du0, dlam=dlam)


@pytest.mark.parametrize("slices,kern", [(4, "pairs8"), (16, "pairs4"), (3, "one_angle")])
def test_unrolled_gradients_launch_paths(oracle_128, slices, kern):
    """The reverse sweep on the launch paths of the large differentiation
    workload: R_h^* split into angle slices (the sweep's backprojection with
    its base image summed by the combine pass), the mirror pairs on 32 x 64
    tiles and the one-angle kernel.  u_K, dL/du0 and dL/dlambda against the
    oracle's reverse mode (1e-5, 1e-4, 1e-4)."""
    o = oracle_128
    print("unrolled launch path", slices, kern, flush=True)
    sino = gpu(o["u0"])[None].requires_grad_(True)
    lt = torch.tensor(o["lam"], device=DEV, requires_grad=True)
    launch = ct.Launch(bp_slices=slices, bp_kernel=kern)
    u = ct.unrolled_pd(o["plan"], sino, lt, [ct.pack_mask(o["mask"])], [gpu(o["bound"])],
                       K=o["K"], every=4, beta=o["beta"], c=o["c"], launch=launch)
    ((u[0] - gpu(o["truth"])) ** 2).mean().backward()
    assert rel(host(u[0]), o["uK"]) <= 1e-5
    assert rel(host(sino.grad[0]), o["du0"]) <= 1e-4
    assert float(lt.grad) == pytest.approx(o["dlam"], rel=1e-4)


def test_unrolled_lambda_fd_large_slice():
    """A 1024^2 x 1440 x 1536 slice (the differentiation workload's size; 6
    unrolled iterations, checkpoints every 3, 4 angle slices on 32 x 64 pair
    tiles): the reverse sweep's dL/dlambda agrees with a central difference
    of the GPU map in lambda to 5 %.  The data are the GPU projection of the
    workload's phantom plus 1 % noise (a GPU-to-GPU check; no oracle).
    lambda = 2000 (lambda~ = lambda / beta^2 ~ 1.4e-3 at this size): large
    enough that the TV term moves the iterates and the loss by far more than
    FP32 rounding within 6 iterations (at the workload's 0.01 the change of
    the loss over the difference step is below its rounding)."""
    print("unrolled fd 1024", flush=True)
    w = synth.workload("C4")
    n, N, M = w.n, w.n_angles, w.n_bins
    plan = ct.Plan(n, N, M)
    clean = plan.radon_fwd(gpu(w.phantom))
    tissue_max = float(plan.radon_fwd(gpu(w.tissue)).max())
    sino = (clean + w.noise_level * tissue_max * gpu(w.noise))[None].contiguous()
    tr = gpu(w.phantom)
    lam, K = 2000.0, 6
    launch = ct.Launch(bp_slices=4, bp_kernel="pairs8")
    probe = ct.Solver(plan, sino[0], lam, launch=launch)
    opts = dict(beta=probe.info()["beta"], c=probe.info()["c"], launch=launch)
    del probe

    def loss(lv, grad=False):
        lt = torch.tensor(lv, device=DEV, requires_grad=grad)
        u = ct.unrolled_pd(plan, sino, lt, K=K, every=3, **opts)
        L = ((u[0] - tr) ** 2).double().mean()
        if grad:
            L.backward()
            return float(L.detach()), float(lt.grad)
        return float(L)

    _, an = loss(lam, True)
    d = 5e-2 * lam
    fd = (loss(lam + d) - loss(lam - d)) / (2 * d)
    print("dL/dlambda reverse %.6e, central difference %.6e" % (an, fd), flush=True)
    assert np.isfinite(an) and an != 0.0
    assert an == pytest.approx(fd, rel=5e-2)
