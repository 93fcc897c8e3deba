"""The largest geometry: 2048^2 image, 2880 angles, 3072 bins, 4 metal discs.

Full-size parity is checked where the oracle can evaluate outputs one by one
(sampled bins of R_h, sampled pixels of R_h^*, the resolvent-side identities
of one iteration at sampled bins and pixels) and through properties that hold
at any size (adjointness, mass per angle, M^{-1} against a full FP64 FFT,
finite and decreasing records)."""
import numpy as np
import pytest
import torch

import synth
from oracle import geometry, precond, prox, radon, tv

pytestmark = pytest.mark.gpu

ct = pytest.importorskip("paper_1810_03275_amd")

DEV = torch.device("cuda")
n, N, M = 2048, 2880, 3072


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def gpu(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(DEV)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


@pytest.fixture(scope="module")
def plan():
    return ct.Plan(n, N, M)


def test_c5_projectors_sampled(plan):
    print("c5 projectors", flush=True)
    g = geometry.Geometry(n, N, M)
    rng = np.random.default_rng(21)
    x = rng.uniform(0, 1, (n, n)).astype(np.float32).astype(np.float64)
    y = rng.uniform(-1, 1, (N, M)).astype(np.float32).astype(np.float64)
    fx = host(plan.radon_fwd(gpu(x)))
    by = host(plan.radon_adj(gpu(y)))
    pix = [(int(j), int(i)) for j, i in rng.integers(0, n, (16, 2))] + [(0, 0), (n - 1, n - 1)]
    assert rel([by[j, i] for j, i in pix], radon.radon_adj_at(g, y, pix)) <= 1e-5
    bins = [(int(l), int(k)) for l, k in zip(rng.integers(0, N, 24), rng.integers(200, 2872, 24))]
    bins += [(0, M // 2), (N // 4, M // 2), (N - 1, 100)]
    assert rel([fx[l, k] for l, k in bins], radon.radon_fwd_at(g, x, bins)) <= 1e-5
    lhs, rhs = np.sum(fx * y), np.sum(x * by)
    assert abs(lhs - rhs) <= 2e-6 * np.linalg.norm(fx) * np.linalg.norm(y)
    assert np.allclose(fx.sum(axis=1), x.sum(), rtol=5e-6)


def test_c5_preconditioner_full():
    print("c5 precond", flush=True)
    rng = np.random.default_rng(22)
    y = rng.standard_normal((n, n)).astype(np.float32).astype(np.float64)
    pc = ct.Precond(n, 1.0, 1.0 / np.sqrt(8.0), 2.0, 0.3)
    got = host(pc.apply(gpu(y)))
    ref = precond.precond_inverse(y, 1.0, 1.0 / np.sqrt(8.0), 2.0, 0.3)
    assert rel(got, ref) <= 1e-5


def test_c5_iterations(plan):
    """20 iterations of the C5 recipe: records finite (the gap record is not
    sign-definite, so only its finiteness is a property); one more
    iteration checked against the oracle at sampled bins (sinogram-side
    resolvent fused into R_h) and sampled pixels (TV side)."""
    print("c5 iterations", flush=True)
    w = synth.workload("C5", iters=20)
    g = geometry.Geometry(n, N, M)
    tissue = plan.radon_fwd(gpu(w.tissue))
    clean = plan.radon_fwd(gpu(w.phantom))
    metal = plan.radon_fwd(gpu(w.metal.astype(np.float32)))
    u0 = clean + w.noise_level * float(tissue.max()) * gpu(w.noise)
    mask = metal > 0
    assert bool(mask.any())
    bound = torch.where(mask, 0.95 * tissue, torch.zeros_like(tissue))
    mb = ct.pack_mask(mask)
    sv = ct.Solver(plan, u0, w.alpha, mb, bound)
    inf = sv.info()
    sv.step(10)
    r10 = sv.gap()
    sv.step(10)
    r20 = sv.gap()
    assert np.all(np.isfinite(r10)) and np.all(np.isfinite(r20))
    assert r10[4] >= 0 and r20[4] >= 0 and r10[3] > 0   # violation, dual residual
    u, vb1, vb2 = (host(t) for t in sv.export())
    sv.step(1)
    u1, vb1n, vb2n = (host(t) for t in sv.export())
    sig, tau = 1.0, 1.0 / np.sqrt(8.0)
    beta = inf["beta"]
    # sinogram side at sampled bins: vb1' = P1(vb1 + 2 sigma r) - sigma r, r = A u'
    rng = np.random.default_rng(23)
    m_host = host(mask.float()) > 0.5
    on = np.argwhere(m_host)
    bins = [tuple(b) for b in on[rng.integers(0, len(on), 12)]]
    bins += [(int(l), int(k)) for l, k in zip(rng.integers(0, N, 12), rng.integers(300, 2772, 12))]
    r = radon.radon_fwd_at(g, u1, bins) / beta
    u0h, bh = host(u0), host(bound)
    for q, (l, k) in enumerate(bins):
        qv = vb1[l, k] + 2.0 * sig * r[q]
        if m_host[l, k]:
            y = min(qv - sig * bh[l, k] / beta, 0.0)
        else:
            y = (qv - sig * u0h[l, k] / beta) / (1.0 + sig)
        ref = y - sig * r[q]
        assert vb1n[l, k] == pytest.approx(ref, rel=1e-4, abs=1e-6 * max(1.0, abs(ref)))
    # TV side at sampled pixels: vb2' = proj(vb2 + 2 sigma tau grad u') - sigma tau grad u'
    gr = tv.grad(u1, 1.0)
    rad = inf["lam_t"] / tau
    for j, i in rng.integers(1, n - 1, (24, 2)):
        qv = vb2[:, j, i] + 2.0 * sig * tau * gr[:, j, i]
        wv = prox.tv_project(qv.reshape(2, 1, 1), rad).reshape(2)
        ref = wv - sig * tau * gr[:, j, i]
        np.testing.assert_allclose(vb2n[:, j, i], ref, rtol=1e-4, atol=1e-6 * rad)
