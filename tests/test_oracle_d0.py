"""Pins of the oracle's metal-trace estimate (no GPU): the dilation equals the
library's binary dilation with a disk, a single pixel at hand-computed bin
positions reaches exactly the bins its two weights reach, the estimate grows
with the marked set, and on a phantom it contains the true metal trace."""
import math

import numpy as np
import pytest
import scipy.ndimage as ndi

from oracle import d0, geometry, radon


@pytest.mark.parametrize("r", [0, 1, 2, 5])
def test_dilate_matches_library_disk(r):
    rng = np.random.default_rng(r)
    marked = rng.random((23, 23)) > 0.97
    yy, xx = np.mgrid[-r:r + 1, -r:r + 1]
    disk = xx * xx + yy * yy <= r * r
    want = ndi.binary_dilation(marked, structure=disk) if r > 0 else marked
    assert np.array_equal(d0.dilate(marked, r), want)


def test_single_pixel_axis_angles_by_hand():
    # n = 8, M = 9, h = ds = 1: pixel column i sits at x = i - 3.5, i.e. bin
    # coordinate t = i + 0.5 at theta = 0, so it splits 1/2, 1/2 between bins
    # i and i + 1; at theta = pi/2 row j does the same between bins j and j + 1.
    g = geometry.Geometry(8, 2, 9, thetas=(0.0, math.pi / 2))
    chi = np.zeros((8, 8))
    j0, i0 = 2, 5
    chi[j0, i0] = 1.0
    proj, mask = d0.trace(g, chi, 0.25)
    want = np.zeros((2, 9))
    want[0, i0] = want[0, i0 + 1] = 0.5
    want[1, j0] = want[1, j0 + 1] = 0.5
    assert np.allclose(proj, want, atol=1e-14)
    assert np.array_equal(mask, want > 0.25)
    # above the common weight nothing is reached
    assert not d0.trace(g, chi, 0.5)[1].any()


def test_single_pixel_weights_per_angle():
    # every angle: at most two adjacent bins, weights summing to 1 (pixel well
    # inside the detector), D0 = the bins whose weight exceeds kappa
    g = geometry.Geometry(16, 37, 24)
    chi = np.zeros((16, 16))
    chi[9, 4] = 1.0
    proj, mask = d0.trace(g, chi, 0.1)
    for l in range(g.n_angles):
        nz = np.flatnonzero(proj[l] > 0)
        assert 1 <= len(nz) <= 2 and (len(nz) == 1 or nz[1] == nz[0] + 1)
        assert abs(proj[l].sum() - 1.0) < 1e-12
        assert np.array_equal(np.flatnonzero(mask[l]), np.flatnonzero(proj[l] > 0.1))


def test_estimate_grows_with_the_marked_set():
    g = geometry.Geometry(20, 30, 32)
    rng = np.random.default_rng(4)
    a = rng.random((20, 20)) > 0.98
    b = rng.random((20, 20)) > 0.98
    _, _, ma = d0.estimate_d0(g, a.astype(float), 0.5, 1, 1e-3)
    _, _, mab = d0.estimate_d0(g, (a | b).astype(float), 0.5, 1, 1e-3)
    assert np.all(mab[ma])
    assert mab.sum() >= ma.sum()


def test_estimate_contains_the_true_metal_trace():
    # tissue disc of density 1, metal disc of density 20: thresholding the
    # true image between the two and dilating covers the metal, so its trace
    # is inside the estimate; the estimate stays a small part of the sinogram
    g = geometry.Geometry(48, 60, 72)
    yy, xx = np.mgrid[0:48, 0:48] - 23.5
    tissue = (xx * xx + yy * yy <= 20 ** 2).astype(float)
    metal = ((xx - 6) ** 2 + (yy + 4) ** 2 <= 3 ** 2).astype(float)
    u = tissue + 19.0 * metal
    kappa = 1e-3
    chi, proj, est = d0.estimate_d0(g, u, 5.0, 5, kappa)
    assert np.all(chi[metal > 0])
    true_trace = radon.radon_fwd(g, metal) > kappa
    assert np.all(est[true_trace])
    assert est.sum() < 0.5 * est.size


def test_bound_from_data():
    u0 = np.arange(6.0).reshape(2, 3)
    m = np.array([[True, False, True], [False, True, False]])
    assert np.array_equal(d0.bound_from_data(u0, m, 0.8), np.where(m, 0.8 * u0, 0.0))
