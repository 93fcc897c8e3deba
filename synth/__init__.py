"""Seeded synthetic inputs for TV-regularized CT reconstruction with metal.

This module draws random numbers and rasterizes simple shapes. It holds none
of the reconstruction method's arithmetic: no projector, no differences, no
Fourier multiplier, no prox.  Both the FP64 oracle (through the tests) and the
GPU path (through the tests and the benchmark) take their inputs from here, so
that the two sides see bit-identical phantoms, noise draws and start vectors.

What is generated (the stand-in for the thesis' Shepp-Logan and metal
experiments of chapter 5, whose parameter tables are not reproduced):

* a tissue phantom: a sum of randomly placed ellipses of constant density,
  sampled at pixel centres in normalized coordinates where the image spans
  [-1, 1]^2 (additive densities);
* metal discs: radius uniform in [8, 20] pixels, centres uniform in the disc of
  normalized radius 0.5, non-overlapping by rejection sampling; disc pixels
  take 20 times the tissue maximum;
* an N x M array of i.i.d. standard normal draws, scaled by the caller into
  detector noise once the caller has projected the phantom;
* standard normal start images for the two power iterations.

The caller combines these with its own projector R_h:
  u0 = R_h P + p * max(R_h P_tissue) * z  off the metal trace,
  D0 = {(l, k) : (R_h 1_metal)[l, k] > 0},  C = 0.95 * R_h P_tissue on D0.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "Workload", "workload", "ellipse_params", "rasterize_ellipses",
    "metal_discs", "disc_mask", "WORKLOADS", "batched_shapes",
]


@dataclasses.dataclass
class Workload:
    """One slice's synthetic inputs and its solver settings."""
    name: str
    n: int            # image side (pixels), grid spacing h = 1
    n_angles: int     # N, angles pi*l/N on [0, pi)
    n_bins: int       # M, detector bins of width ds = 1
    tissue: np.ndarray          # (n, n) float64, tissue phantom
    metal: np.ndarray           # (n, n) bool, metal pixels
    metal_value: float          # density written at metal pixels
    noise: np.ndarray           # (N, M) float64 standard normal draws
    noise_level: float          # p: noise std is p * max(R_h tissue)
    alpha: float                # regularization weight (unnormalized lambda)
    iters: int                  # iteration count the workload is run for
    start_norm: np.ndarray      # (n, n) start image for the ||R_h|| power iteration
    start_precond: np.ndarray   # (n, n) start image for the c power iteration
    seed: int

    @property
    def phantom(self) -> np.ndarray:
        """Tissue with metal pixels overwritten by the metal density."""
        p = self.tissue.copy()
        p[self.metal] = self.metal_value
        return p


def ellipse_params(rng: np.random.Generator, count: int) -> np.ndarray:
    """(count, 6) rows: cx, cy, semi-axis a, semi-axis b, angle, density.

    Centres U[-0.6, 0.6]^2, semi-axes U[0.05, 0.4], angle U[0, pi),
    density U[0.1, 1], all in normalized image coordinates.
    """
    cx = rng.uniform(-0.6, 0.6, count)
    cy = rng.uniform(-0.6, 0.6, count)
    a = rng.uniform(0.05, 0.4, count)
    b = rng.uniform(0.05, 0.4, count)
    phi = rng.uniform(0.0, math.pi, count)
    rho = rng.uniform(0.1, 1.0, count)
    return np.stack([cx, cy, a, b, phi, rho], axis=1)


def _normalized_centres(n: int, supersample: int = 1) -> np.ndarray:
    """Normalized coordinates of (sub-)pixel centres along one axis.

    Pixel i has centre (i - (n-1)/2) / (n/2); with s x s supersampling the
    sub-samples sit at the centres of the s^2 equal sub-squares of the pixel.
    """
    s = supersample
    sub = (np.arange(n * s) + 0.5) / s - 0.5          # pixel units, centre of pixel i at i
    return (sub - (n - 1) / 2.0) / (n / 2.0)


def rasterize_ellipses(params: np.ndarray, n: int, supersample: int = 1) -> np.ndarray:
    """Additive ellipse image (n, n), row index j = y, column index i = x.

    With supersample s > 1 each pixel holds the mean over s x s sub-samples,
    an approximation of the area-weighted density.
    """
    c = _normalized_centres(n, supersample)
    X, Y = np.meshgrid(c, c, indexing="xy")   # X varies along columns (i), Y along rows (j)
    img = np.zeros_like(X)
    for cx, cy, a, b, phi, rho in params:
        dx, dy = X - cx, Y - cy
        xr = dx * math.cos(phi) + dy * math.sin(phi)
        yr = -dx * math.sin(phi) + dy * math.cos(phi)
        img += rho * ((xr / a) ** 2 + (yr / b) ** 2 <= 1.0)
    if supersample > 1:
        s = supersample
        img = img.reshape(n, s, n, s).mean(axis=(1, 3))
    return img


def metal_discs(rng: np.random.Generator, count: int, n: int,
                max_tries: int = 10000, radius_scale: float = 1.0) -> np.ndarray:
    """(count, 3) rows: centre x, centre y (pixel units from the image centre), radius.

    Radii U[8, 20] px (times radius_scale, used only to shrink a workload to a
    test-sized image); centres uniform in the disc of normalized radius 0.5
    (i.e. n/4 pixels); discs do not overlap (rejection sampling).
    """
    discs: list[tuple[float, float, float]] = []
    tries = 0
    rmax_centre = 0.5 * n / 2.0
    while len(discs) < count:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("could not place non-overlapping metal discs")
        r = radius_scale * rng.uniform(8.0, 20.0)
        rad = rmax_centre * math.sqrt(rng.uniform(0.0, 1.0))
        ang = rng.uniform(0.0, 2.0 * math.pi)
        cx, cy = rad * math.cos(ang), rad * math.sin(ang)
        if all(math.hypot(cx - x, cy - y) > r + rr + 1.0 for x, y, rr in discs):
            discs.append((cx, cy, r))
    return np.array(discs, dtype=np.float64).reshape(count, 3)


def disc_mask(discs: np.ndarray, n: int) -> np.ndarray:
    """Boolean (n, n) mask of pixels whose centre lies in any disc."""
    c = np.arange(n) - (n - 1) / 2.0
    X, Y = np.meshgrid(c, c, indexing="xy")
    m = np.zeros((n, n), dtype=bool)
    for cx, cy, r in discs:
        m |= (X - cx) ** 2 + (Y - cy) ** 2 <= r * r
    return m


# name -> (n, N, M, ellipses, metal discs, noise p, alpha, iterations)
WORKLOADS = {
    "C1": (64, 90, 96, 6, 0, 0.01, 0.01, 200),
    "C2": (512, 720, 768, 6, 2, 0.005, 0.005, 500),
    "C4": (1024, 1440, 1536, 6, 0, 0.01, 0.01, 50),
    "C5": (2048, 2880, 3072, 6, 4, 0.005, 0.005, 1000),
}


def _make(name: str, n: int, N: int, M: int, n_ell: int, n_metal: int,
          p: float, alpha: float, iters: int, seed: int) -> Workload:
    rng = np.random.default_rng(seed)
    tissue = rasterize_ellipses(ellipse_params(rng, n_ell), n)
    if n_metal > 0:
        scale = min(1.0, n / 512.0)
        metal = disc_mask(metal_discs(rng, n_metal, n, radius_scale=scale), n)
    else:
        metal = np.zeros((n, n), dtype=bool)
    metal_value = 20.0 * float(tissue.max())
    noise = rng.standard_normal((N, M))
    start_norm = rng.standard_normal((n, n))
    start_precond = rng.standard_normal((n, n))
    return Workload(name, n, N, M, tissue, metal, metal_value, noise, p, alpha,
                    iters, start_norm, start_precond, seed)


def workload(name: str, slice_index: int = 0, *, n: int | None = None,
             n_angles: int | None = None, n_bins: int | None = None,
             iters: int | None = None) -> Workload:
    """Seeded workload by name ("C1", "C2", "C4", "C5"), seed 1000*config + slice.

    Keyword overrides shrink a workload to a test-sized shape with the same
    recipe (phantom statistics, metal count, noise level, alpha).
    """
    base = WORKLOADS[name]
    n0, N0, M0, n_ell, n_metal, p, alpha, it = base
    cfg_index = int(name[1:])
    seed = 1000 * cfg_index + slice_index
    n = n0 if n is None else n
    N = N0 if n_angles is None else n_angles
    M = M0 if n_bins is None else n_bins
    it = it if iters is None else iters
    return _make(name, n, N, M, n_ell, n_metal, p, alpha, it, seed)


def batched_shapes(count: int = 64, seed: int = 3000,
                   sizes=(256, 384, 512, 768, 1024)) -> list[tuple[int, int, int, int]]:
    """Uneven batched slices: (n, N, M, metal discs) per slice.

    n is drawn from `sizes` ({256, 384, 512, 768, 1024} for the full batch);
    N = round(1.4 n); M = 1.5 n; 0-3 metal discs.
    """
    rng = np.random.default_rng(seed)
    sizes = np.array(sizes)
    out = []
    for _ in range(count):
        n = int(rng.choice(sizes))
        out.append((n, int(round(1.4 * n)), int(1.5 * n), int(rng.integers(0, 4))))
    return out


def batched_workload(slice_index: int, shape: tuple[int, int, int, int],
                     iters: int = 300) -> Workload:
    """One slice of the uneven batch, seed 3000 + slice."""
    n, N, M, n_metal = shape
    return _make("C3", n, N, M, 6, n_metal, 0.005, 0.005, iters, 3000 + slice_index)
