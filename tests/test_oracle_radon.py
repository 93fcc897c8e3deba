"""Pins of the oracle's discrete Radon pair (thesis §3.1) against facts fixed
by the thesis and by mathematics, not against the oracle's own formula."""
import math

import numpy as np
import pytest

from oracle import geometry, power, radon

GEOMS = [
    geometry.Geometry(8, 6, 12),
    geometry.Geometry(9, 7, 13),            # odd n, odd M
    geometry.Geometry(12, 10, 20, h=1.0, ds=1.3),
    geometry.Geometry(16, 12, 24, h=0.8, ds=1.0),
]


@pytest.mark.parametrize("g", GEOMS)
def test_adjoint_identity(g):
    """R_h is defined as the transpose of R_h^* (§3.1): <R x, y> = <x, R^* y>."""
    rng = np.random.default_rng(1)
    x = rng.standard_normal((g.n, g.n))
    y = rng.standard_normal((g.n_angles, g.n_bins))
    lhs = np.sum(radon.radon_fwd(g, x) * y)
    rhs = np.sum(x * radon.radon_adj(g, y))
    scale = np.linalg.norm(radon.radon_fwd(g, x)) * np.linalg.norm(y)
    assert abs(lhs - rhs) <= 1e-12 * scale


@pytest.mark.parametrize("g", GEOMS[:3])
def test_scatter_gather_and_bruteforce_matrix(g):
    """Three independent forms of the same sums: literal scatter, per-bin
    gather, and a dense matrix built pixel by pixel with scalar math."""
    rng = np.random.default_rng(2)
    x = rng.standard_normal((g.n, g.n))
    y = rng.standard_normal((g.n_angles, g.n_bins))
    fwd = radon.radon_fwd(g, x)
    assert np.max(np.abs(radon.radon_fwd_gather(g, x) - fwd)) <= 1e-13 * np.abs(fwd).max()
    A = radon.radon_matrix(g)
    assert np.max(np.abs(A @ x.ravel() - fwd.ravel())) <= 1e-12
    assert np.max(np.abs(A.T @ y.ravel() - radon.radon_adj(g, y).ravel())) <= 1e-12
    # each column (pixel) has weights summing to one per angle when inside
    col = A.reshape(g.n_angles, g.n_bins, g.n * g.n).sum(axis=1)
    assert np.all(col <= 1.0 + 1e-12) and np.all(col >= -1e-15)


def test_weights_are_linear_interpolation():
    """A pixel projecting a fraction alpha past bin centre k is split as
    (1 - alpha) to k and alpha to k+1: the value interpolated at t by R^* is
    the linear interpolant of the detector row (continuity in t, §3.1 text
    and figure caption)."""
    g = geometry.Geometry(1, 1, 8)     # one pixel at the origin, theta = 0: t = 3.5
    v = np.arange(8, dtype=np.float64)[None, :] ** 2
    got = radon.radon_adj(g, v)[0, 0]
    assert got == pytest.approx(0.5 * 9 + 0.5 * 16)
    g2 = geometry.Geometry(2, 1, 8)    # pixels at x = -0.5, 0.5: t = 3.0, 4.0
    u = np.zeros((2, 2))
    u[0, 0] = 1.0                      # x = -0.5 -> t = 3.0 exactly: all weight on bin 3
    assert radon.radon_fwd(g2, u)[0].tolist() == [0, 0, 0, 1, 0, 0, 0, 0]


def test_mass_conservation_and_backprojection_of_ones():
    """With every pixel projecting strictly inside the detector, each angle's
    weights sum to one: sum_k (R u)[l, k] = sum u, and R^* 1 = N."""
    g = geometry.Geometry(20, 14, 32)   # 20 * sqrt(2) + 2 < 32
    rng = np.random.default_rng(3)
    u = rng.uniform(0, 1, (20, 20))
    s = radon.radon_fwd(g, u)
    assert np.allclose(s.sum(axis=1), u.sum(), rtol=0, atol=1e-11)
    assert np.allclose(radon.radon_adj(g, np.ones((14, 32))), 14.0, atol=1e-12)


def test_rotation_by_90_degrees():
    """Rotating the image by +90 degrees shifts the sinogram by N/2 angles;
    rows that wrap past pi are reversed in s (bins k -> M-1-k)."""
    g = geometry.Geometry(10, 16, 20)
    rng = np.random.default_rng(4)
    u = rng.standard_normal((10, 10))
    n = g.n
    # u'(x, y) = u(y, -x): pixel (i, j) moves to (i', j') = (n-1-j, i)
    ur = np.zeros_like(u)
    for j in range(n):
        for i in range(n):
            ur[i, n - 1 - j] = u[j, i]
    s = radon.radon_fwd(g, u)
    sr = radon.radon_fwd(g, ur)
    h = g.n_angles // 2
    assert np.allclose(sr[h:], s[:h], atol=1e-9)
    assert np.allclose(sr[:h], s[h:, ::-1], atol=1e-9)


def _ellipse_projection(s, theta, cx, cy, a, b, phi, rho):
    """Line integral of a constant-density ellipse at (theta, s): the chord
    length 2ab sqrt(q^2 - s'^2)/q^2, q^2 = a^2 cos^2(theta-phi) + b^2 sin^2(theta-phi)."""
    q2 = (a * math.cos(theta - phi)) ** 2 + (b * math.sin(theta - phi)) ** 2
    sp = s - (cx * math.cos(theta) + cy * math.sin(theta))
    val = np.where(sp ** 2 < q2, 2 * a * b * np.sqrt(np.maximum(q2 - sp ** 2, 0)) / q2, 0.0)
    return rho * val


def _hat_smoothed(s, theta, e, ds=1.0, quad=64):
    """The closed form convolved with the detector hat function of width ds
    (what an exact line-integral transform followed by linear splitting gives)."""
    x = (np.arange(quad) + 0.5) / quad * 2 - 1       # (-1, 1)
    w = (1 - np.abs(x)) * (2.0 / quad)
    out = np.zeros_like(s)
    for xi, wi in zip(x, w):
        out += wi * _ellipse_projection(s + xi * ds, theta, *e)
    return out


def test_ellipse_closed_form_converges():
    """R_h of an area-sampled ellipse approaches the textbook line integral of
    the ellipse (with the detector hat blur) at rate O(h).  This pins the
    angle convention s = x cos theta + y sin theta, the bin offset and the
    interpolation weights.  N = 22 avoids theta = pi/4, where pixel centres
    project onto a lattice of spacing h/sqrt(2) and the linear splitting
    leaves an O(1) comb pattern that does not vanish with h."""
    from synth import rasterize_ellipses
    e_norm = (0.21, -0.13, 0.55, 0.3, 0.7, 1.0)   # normalized units, image = [-1,1]^2
    errs = []
    for n in (32, 64, 128):
        N, M = 22, int(1.5 * n)
        g = geometry.Geometry(n, N, M)
        img = rasterize_ellipses(np.array([e_norm]), n, supersample=8)
        sino = radon.radon_fwd(g, img)
        half = n / 2.0                                 # normalized -> pixel units
        e_px = (e_norm[0] * half, e_norm[1] * half, e_norm[2] * half, e_norm[3] * half, e_norm[4], 1.0)
        ref = np.stack([_hat_smoothed(g.bin_centres(), th, e_px, quad=128) for th in g.angles()])
        errs.append(np.linalg.norm(sino - ref) / np.linalg.norm(ref))
    assert errs[-1] < 0.005
    assert errs[1] < 0.6 * errs[0] and errs[2] < 0.6 * errs[1]


def test_swapped_convention_fails_ellipse_pin():
    """The ellipse pin detects a transposed image (x/y swap)."""
    from synth import rasterize_ellipses
    n = 64
    g = geometry.Geometry(n, 22, 96)
    e_norm = (0.21, -0.13, 0.55, 0.3, 0.7, 1.0)
    img = rasterize_ellipses(np.array([e_norm]), n, supersample=8)
    half = n / 2.0
    e_px = (e_norm[0] * half, e_norm[1] * half, e_norm[2] * half, e_norm[3] * half, e_norm[4], 1.0)
    ref = np.stack([_hat_smoothed(g.bin_centres(), th, e_px) for th in g.angles()])
    good = np.linalg.norm(radon.radon_fwd(g, img) - ref) / np.linalg.norm(ref)
    bad = np.linalg.norm(radon.radon_fwd(g, img.T) - ref) / np.linalg.norm(ref)
    assert bad > 10 * good


def test_norm_bound_and_constants_not_annihilated():
    """||R_h|| <= sqrt(2N(sqrt(2) n + 1)) for ds < h sqrt(2) (lemma in §3.1);
    R_h 1 != 0."""
    for g in (geometry.Geometry(8, 6, 12), geometry.Geometry(10, 9, 15, ds=1.2)):
        A = radon.radon_matrix(g)
        smax = np.linalg.svd(A, compute_uv=False)[0]
        assert smax <= math.sqrt(2 * g.n_angles * (math.sqrt(2) * g.n + 1))
        assert np.linalg.norm(A @ np.ones(g.n * g.n)) > 0
        rng = np.random.default_rng(5)
        est = power.radon_norm(lambda u: radon.radon_fwd(g, u), lambda v: radon.radon_adj(g, v),
                               rng.standard_normal((g.n, g.n)), iters=300)
        assert est == pytest.approx(smax, rel=1e-6)


def test_impulse_response_inverse_distance():
    """R^* R of a point is approximately N / (pi r) at distance r (the
    continuous R^* R is convolution with 1/|x|, §1.2.2 lemma, with N angles
    spread over pi)."""
    n, N = 64, 180
    g = geometry.Geometry(n, N, 96)
    d = np.zeros((n, n))
    d[32, 32] = 1.0
    k = radon.radon_adj(g, radon.radon_fwd(g, d))
    x = np.arange(n) - 32
    X, Y = np.meshgrid(x, x)
    r = np.hypot(X, Y)
    for r0 in (6, 9, 12, 15):
        sel = (r > r0 - 0.5) & (r <= r0 + 0.5)
        ratio = np.mean(k[sel] * np.pi * r[sel] / N)
        assert ratio == pytest.approx(1.0, abs=0.1)


def test_reversed_weights_fail_ellipse_pin(monkeypatch):
    """Planting the literal printed weight orientation (alpha to floor(t),
    1 - alpha to floor(t)+1) in the oracle makes the closed-form pin fail,
    so the pin decides that reading."""
    from synth import rasterize_ellipses
    n = 64
    g = geometry.Geometry(n, 22, 96)
    e_norm = (0.21, -0.13, 0.55, 0.3, 0.7, 1.0)
    img = rasterize_ellipses(np.array([e_norm]), n, supersample=8)
    half = n / 2.0
    e_px = (e_norm[0] * half, e_norm[1] * half, e_norm[2] * half, e_norm[3] * half, e_norm[4], 1.0)
    ref = np.stack([_hat_smoothed(g.bin_centres(), th, e_px) for th in g.angles()])
    good = np.linalg.norm(radon.radon_fwd(g, img) - ref) / np.linalg.norm(ref)
    orig = radon._floor_and_weight

    def reversed_weights(t):
        k, a = orig(t)
        return k, 1.0 - a
    monkeypatch.setattr(radon, "_floor_and_weight", reversed_weights)
    bad = np.linalg.norm(radon.radon_fwd(g, img) - ref) / np.linalg.norm(ref)
    assert bad > 5 * good


# ---------------------------------------------------------------------------
# The one-by-one evaluators behind the full-size GPU spot checks.  They are
# pinned here against the whole-array projector pair, which the brute-force
# matrix and the adjoint identity pin above (§3.1: R_h is the transpose of
# R_h^*), at every pixel and bin of small geometries, explicit angles
# included.

SAMPLED_GEOMS = [
    geometry.Geometry(10, 8, 16),
    geometry.Geometry(9, 7, 13, h=1.0, ds=1.3),                         # odd n and M, ds != h
    geometry.Geometry(12, 5, 20, thetas=(0.3, 2.9, -1.1, 4.0, 1.5707963267948966)),
]


def _all_pixels(g):
    return [(j, i) for j in range(g.n) for i in range(g.n)]


def _all_bins(g):
    return [(l, k) for l in range(g.n_angles) for k in range(g.n_bins)]


def _adj_at_pin(g, adj_at, seed=31):
    rng = np.random.default_rng(seed)
    v = rng.standard_normal((g.n_angles, g.n_bins))
    ref = radon.radon_adj(g, v).ravel()
    got = adj_at(g, v, _all_pixels(g))
    return float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))


def _fwd_at_pin(g, fwd_at, seed=32):
    rng = np.random.default_rng(seed)
    u = rng.standard_normal((g.n, g.n))
    ref = radon.radon_fwd(g, u).ravel()
    got = fwd_at(g, u, _all_bins(g))
    return float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))


@pytest.mark.parametrize("g", SAMPLED_GEOMS)
def test_sampled_evaluators_match_whole_arrays(g):
    """radon_adj_at / radon_fwd_at equal the whole-array R_h^* / R_h at every
    pixel and every bin (bins are visited angle by angle, then in a shuffled
    order so that the per-angle cache is refilled)."""
    assert _adj_at_pin(g, radon.radon_adj_at) <= 1e-13
    assert _fwd_at_pin(g, radon.radon_fwd_at) <= 1e-13
    rng = np.random.default_rng(33)
    u = rng.standard_normal((g.n, g.n))
    bins = _all_bins(g)
    order = rng.permutation(len(bins))
    got = radon.radon_fwd_at(g, u, [bins[q] for q in order])
    assert np.max(np.abs(got - radon.radon_fwd(g, u).ravel()[order])) <= 1e-12


def _fwd_at_offbyone(g, u, bins):
    # planted mistake: the alpha term taken from the strip of bin k itself
    out = np.zeros(len(bins))
    for q, (l, k) in enumerate(bins):
        t = g.bin_coordinate(l)
        kk = np.floor(t)
        a = t - kk
        out[q] = np.sum(((1.0 - a) * u)[kk == k]) + np.sum((a * u)[kk == k])
    return out


def _adj_at_swapped(g, v, pixels):
    # planted mistake: the weights of the two bins exchanged
    out = np.zeros(len(pixels))
    for q, (j, i) in enumerate(pixels):
        for l in range(g.n_angles):
            t = g.bin_coordinate_scalar(i, j, l)
            k = math.floor(t)
            a = t - k
            if 0 <= k < g.n_bins:
                out[q] += a * v[l, k]
            if 0 <= k + 1 < g.n_bins:
                out[q] += (1.0 - a) * v[l, k + 1]
    return out


def _default_angles(fn):
    # planted mistake: the explicit angles ignored (theta_l = pi l / N used)
    import dataclasses
    return lambda g, x, idx: fn(dataclasses.replace(g, thetas=None), x, idx)


@pytest.mark.parametrize("mutant,kind", [
    (_fwd_at_offbyone, "fwd"), (_adj_at_swapped, "adj"),
    (_default_angles(radon.radon_fwd_at), "fwd"), (_default_angles(radon.radon_adj_at), "adj"),
])
def test_sampled_evaluator_pin_catches_planted_mistakes(mutant, kind):
    """Each planted mistake in a sampled evaluator fails the pin above on the
    geometry with explicit angles."""
    g = SAMPLED_GEOMS[2]
    err = _fwd_at_pin(g, mutant) if kind == "fwd" else _adj_at_pin(g, mutant)
    assert err > 1e-2


def test_angle_blocks_equal_serial_pair():
    """The angle-block split of the pair (worker processes) gives the serial
    oracle's R_h exactly and its R_h^* to FP64 rounding, explicit angles
    included."""
    from oracle.parallel import AngleBlocks
    for g in (geometry.Geometry(20, 17, 30), SAMPLED_GEOMS[2]):
        ab = AngleBlocks(g, 2)
        try:
            rng = np.random.default_rng(41)
            u = rng.standard_normal((g.n, g.n))
            v = rng.standard_normal((g.n_angles, g.n_bins))
            assert np.array_equal(ab.fwd(u), radon.radon_fwd(g, u))
            ref = radon.radon_adj(g, v)
            assert np.max(np.abs(ab.adj(v) - ref)) <= 1e-13 * np.max(np.abs(ref))
        finally:
            ab.close()
