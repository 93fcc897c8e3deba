"""Metal-trace estimate on the GPU vs the FP64 oracle, through the C ABI.

The dilated indicator is compared bit for bit (the threshold decision is made
on the same FP32 values on both sides); R_h chi to the projector's 1e-5; the
D0 bits exactly wherever the oracle's projection is not within 1e-5 of kappa
(there either decision is correct); the bound to FP32 rounding.
"""
import numpy as np
import pytest
import torch

from oracle import d0, geometry, radon

pytestmark = pytest.mark.gpu

ct = pytest.importorskip("paper_1810_03275_amd")

DEV = torch.device("cuda")


def gpu(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(DEV)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def unpack(mask, M):
    words = host(mask).astype(np.uint32)
    bits = np.unpackbits(words.view(np.uint8), axis=1, bitorder="little").astype(bool)
    return bits[:, :M], bits[:, M:]


def phantom(n, seed, n_metal=2):
    """Tissue disc (density U[0.5, 1]) with small dense discs, plus noise: a
    stand-in for an unconstrained reconstruction with metal."""
    rng = np.random.default_rng(seed)
    yy, xx = np.mgrid[0:n, 0:n] - (n - 1) / 2.0
    u = np.where(xx * xx + yy * yy <= (0.45 * n) ** 2, rng.uniform(0.5, 1.0), 0.0)
    for _ in range(n_metal):
        cx, cy = rng.uniform(-0.25 * n, 0.25 * n, 2)
        r = rng.uniform(0.03 * n, 0.06 * n)
        u = np.where((xx - cx) ** 2 + (yy - cy) ** 2 <= r * r, 20.0, u)
    return (u + 0.3 * rng.standard_normal((n, n))).astype(np.float32)


def check(g, u, thr, r, kappa, u0=None, c0=0.8):
    plan = ct.Plan(g.n, g.n_angles, g.n_bins, g.h, g.ds)
    chi, proj, mask, bound = ct.estimate_d0(plan, gpu(u), thr, r, kappa,
                                            u0=None if u0 is None else gpu(u0), c0=c0)
    chi_o, proj_o, d0_o = d0.estimate_d0(g, u.astype(np.float64), np.float32(thr), r, kappa)
    assert np.array_equal(host(chi), chi_o.astype(np.float32))
    p = host(proj).astype(np.float64)
    den = max(np.linalg.norm(proj_o), 1e-300)
    assert np.linalg.norm(p - proj_o) / den <= 1e-5 or np.linalg.norm(proj_o) == 0
    bits, pad = unpack(mask, g.n_bins)
    assert not pad.any()
    sure = np.abs(proj_o - kappa) > 1e-5
    assert np.array_equal(bits[sure], d0_o[sure])
    if u0 is not None:
        want = d0.bound_from_data(u0.astype(np.float64), bits, c0)
        assert np.allclose(host(bound), want, rtol=1e-6, atol=0)
    return bits, d0_o


@pytest.mark.parametrize("geo,r", [((64, 90, 96), 5), ((50, 37, 70), 3), ((96, 1, 140), 0),
                                   ((40, 33, 64), 16), ((2, 3, 4), 1)],
                         ids=["64x90x96-r5", "ragged-50x37x70-r3", "one-angle-r0", "r16", "tiny"])
def test_d0_estimate_matches_oracle(geo, r):
    n, N, M = geo
    print("d0 estimate", geo, r, flush=True)
    g = geometry.Geometry(n, N, M)
    u = phantom(n, n + r)
    rng = np.random.default_rng(7)
    u0 = rng.uniform(0.0, 5.0, (N, M)).astype(np.float32)
    check(g, u, 5.0, r, 1e-3, u0=u0)


def test_d0_estimate_degenerate_thresholds():
    g = geometry.Geometry(48, 30, 64)
    u = phantom(48, 3)
    bits, _ = check(g, u, 1e6, 5, 1e-3)      # nothing marked: empty D0
    assert not bits.any()
    bits, d0_o = check(g, u, -1e6, 2, 1e-3)  # everything marked: the image's whole trace
    full = radon.radon_fwd(g, np.ones((48, 48))) > 1e-3
    assert np.array_equal(d0_o, full)


def test_d0_estimate_c2_size_contains_true_trace():
    # 512 x 512, 720 angles, 768 bins: the dilated marks match the oracle's
    # dilation exactly and D0 holds the trace of the dense discs
    print("d0 estimate 512x720x768", flush=True)
    n, N, M = 512, 720, 768
    u = phantom(n, 11)
    plan = ct.Plan(n, N, M)
    chi, proj, mask, _ = ct.estimate_d0(plan, gpu(u), 5.0, 5, 1e-3)
    assert np.array_equal(host(chi), d0.dilate(d0.mark(u, np.float32(5.0)), 5).astype(np.float32))
    bits, pad = unpack(mask, M)
    assert not pad.any()
    dense = (u > 5.0).astype(np.float32)
    trace = host(plan.radon_fwd(gpu(dense))) > 1e-3
    assert np.all(bits[trace])
    # sampled bins: the decision where the oracle's projection is clear of kappa
    g = geometry.Geometry(n, N, M)
    rng = np.random.default_rng(5)
    ls = rng.integers(0, N, 24)
    ks = rng.integers(0, M, 24)
    vals = radon.radon_fwd_at(g, host(chi).astype(np.float64), list(zip(ls, ks)))
    for (l, k), v in zip(zip(ls, ks), vals):
        if abs(v - 1e-3) > 1e-5:
            assert bits[l, k] == (v > 1e-3)


def test_d0_estimate_rejects_bad_arguments():
    plan = ct.Plan(32, 10, 48)
    u = gpu(np.zeros((32, 32)))
    with pytest.raises(ct.CtpdError):
        ct.estimate_d0(plan, u, 1.0, 17)
    with pytest.raises(ct.CtpdError):
        ct.estimate_d0(plan, u, 1.0, -1)
    with pytest.raises(ct.CtpdError):
        ct.estimate_d0(plan, u, 1.0, 2, kappa=-1.0)
    with pytest.raises(ct.CtpdError):
        ct.estimate_d0(plan, u, float("nan"), 2)
