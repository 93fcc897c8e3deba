"""Estimate of the metal trace D0 from a reconstruction (thesis, results
chapter, real metal artifacts).  Test infrastructure only (see the package
header).

The thesis marks the sinogram bins affected by metal in four steps, taken
here in its order:
  1. a regular (unconstrained) reconstruction u_rec is computed;
  2. the image pixels where u_rec exceeds a threshold are marked;
  3. the marked set is dilated (by 5 pixels in the thesis' experiment);
  4. the marked set is carried to the sinogram: D0 holds the bins that its
     projection reaches.
The constraint on D0 is then set from the data, C = c0 u0 (c0 = 0.8 there).

Readings (the passage gives the steps, not their exact rules):
  * the dilation by r pixels: the Euclidean disk {(a, b) : a^2 + b^2 <= r^2}
    of pixel offsets; the image has no pixels outside [0, n)^2.
  * the step that carries the marked image areas over to the sinogram maps
    image to sinogram, i.e. R_h of the indicator image chi of the marked
    set.  A bin belongs to D0 when (R_h chi)[l, k] > kappa for a
    small kappa > 0: R_h splits every pixel between two bins with weights
    1 - alpha and alpha that sum to 1, so kappa is the smallest weight with
    which a marked pixel must reach a bin (a threshold of zero would make the
    decision depend on the rounding of weights near 0).
"""
from __future__ import annotations

import numpy as np

from . import radon
from .geometry import Geometry


def disk_offsets(r: int):
    """Pixel offsets (a, b) with a^2 + b^2 <= r^2."""
    return [(a, b) for b in range(-r, r + 1) for a in range(-r, r + 1) if a * a + b * b <= r * r]


def mark(u_rec: np.ndarray, threshold: float) -> np.ndarray:
    """Step 2: pixels whose reconstructed value exceeds the threshold."""
    return np.asarray(u_rec, dtype=np.float64) > float(threshold)


def dilate(marked: np.ndarray, r: int) -> np.ndarray:
    """Step 3: chi[j, i] = 1 iff some marked pixel lies within the disk of
    radius r around (i, j).  Written as the union of shifted copies."""
    marked = np.asarray(marked, dtype=bool)
    n1, n0 = marked.shape
    out = np.zeros_like(marked)
    for a, b in disk_offsets(r):
        # out[j, i] |= marked[j + b, i + a] where that pixel exists
        js = slice(max(0, -b), min(n1, n1 - b))
        is_ = slice(max(0, -a), min(n0, n0 - a))
        jd = slice(max(0, b), min(n1, n1 + b))
        id_ = slice(max(0, a), min(n0, n0 + a))
        out[js, is_] |= marked[jd, id_]
    return out


def trace(g: Geometry, chi: np.ndarray, kappa: float):
    """Step 4: the projection R_h chi and D0 = {R_h chi > kappa}."""
    proj = radon.radon_fwd(g, np.asarray(chi, dtype=np.float64))
    return proj, proj > kappa


def estimate_d0(g: Geometry, u_rec: np.ndarray, threshold: float, r: int, kappa: float):
    """Steps 2-4: (chi, R_h chi, D0)."""
    chi = dilate(mark(u_rec, threshold), r)
    proj, d0 = trace(g, chi, kappa)
    return chi, proj, d0


def bound_from_data(u0: np.ndarray, d0: np.ndarray, c0: float) -> np.ndarray:
    """C = c0 u0 on D0 (zero elsewhere, where the constraint is not used)."""
    return np.where(d0, c0 * np.asarray(u0, dtype=np.float64), 0.0)
