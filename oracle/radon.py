"""Discrete Radon pair R_h^*, R_h (thesis §3.1, "Discretization").

R_h^* (linear backprojection): for every pixel and angle the detector value
at the pixel's bin coordinate t is interpolated linearly between bins
floor(t) and floor(t)+1, and the per-angle values are summed.  R_h is defined
as the transpose of R_h^*: a pixel's value is split between the same two bins
with the same two weights.

Reading of the weights: the printed formula gives weight alpha to bin k and
1 - alpha to bin k + 1 with alpha = t - floor(t), which is discontinuous in t
and contradicts both the text, which names the scheme linear interpolation,
and the figure caption, where a value is shared by the two nearest bins in
proportion to its distance from them.  The oracle uses
standard linear interpolation: weight 1 - alpha to bin floor(t) and alpha to
bin floor(t) + 1.

Reading of the detector edge (silent in the thesis): a bin index outside
[0, M) contributes nothing in R_h^* and receives nothing in R_h.

Three independent forms are provided so that the tests can pin them against
each other: the backprojection gather, the forward projection as the literal
scatter ("splitting" each pixel), and a per-bin gather form of the same sums.
A dense matrix built from scalar loops serves brute-force checks.
"""
from __future__ import annotations

import math

import numpy as np

from .geometry import Geometry


def _floor_and_weight(t: np.ndarray):
    k = np.floor(t)
    return k.astype(np.int64), t - k


def radon_adj(g: Geometry, v: np.ndarray) -> np.ndarray:
    """(R_h^* v)[j, i] = sum_l (1 - alpha) v[l, k] + alpha v[l, k+1]  (§3.1).

    v has shape (N, M); the result has shape (n, n).
    """
    v = np.asarray(v, dtype=np.float64)
    assert v.shape == (g.n_angles, g.n_bins)
    out = np.zeros((g.n, g.n), dtype=np.float64)
    M = g.n_bins
    for l in range(g.n_angles):
        k, a = _floor_and_weight(g.bin_coordinate(l))
        row = v[l]
        in0 = (k >= 0) & (k < M)
        in1 = (k + 1 >= 0) & (k + 1 < M)
        out += np.where(in0, (1.0 - a) * row[np.clip(k, 0, M - 1)], 0.0)
        out += np.where(in1, a * row[np.clip(k + 1, 0, M - 1)], 0.0)
    return out


def radon_fwd(g: Geometry, u: np.ndarray) -> np.ndarray:
    """(R_h u)[l, k]: the transpose of radon_adj, as the literal scatter (§3.1).

    Every pixel u[j, i] adds (1 - alpha) u to bin floor(t) and alpha u to bin
    floor(t) + 1 of angle l.  Result shape (N, M).
    """
    u = np.asarray(u, dtype=np.float64)
    assert u.shape == (g.n, g.n)
    M = g.n_bins
    out = np.zeros((g.n_angles, M), dtype=np.float64)
    uf = u.ravel()
    for l in range(g.n_angles):
        k, a = _floor_and_weight(g.bin_coordinate(l))
        k = k.ravel()
        a = a.ravel()
        m0 = (k >= 0) & (k < M)
        m1 = (k + 1 >= 0) & (k + 1 < M)
        out[l] += np.bincount(k[m0], weights=((1.0 - a) * uf)[m0], minlength=M)[:M]
        out[l] += np.bincount(k[m1] + 1, weights=(a * uf)[m1], minlength=M)[:M]
    return out


def radon_fwd_gather(g: Geometry, u: np.ndarray) -> np.ndarray:
    """R_h u computed bin by bin: bin k of angle l sums (1 - alpha) u over the
    pixels with floor(t) = k and alpha u over those with floor(t) = k - 1.

    O(N M n^2); for small problems only.
    """
    u = np.asarray(u, dtype=np.float64)
    out = np.zeros((g.n_angles, g.n_bins), dtype=np.float64)
    for l in range(g.n_angles):
        k, a = _floor_and_weight(g.bin_coordinate(l))
        for kb in range(g.n_bins):
            out[l, kb] = np.sum(((1.0 - a) * u)[k == kb]) + np.sum((a * u)[k == kb - 1])
    return out


def radon_matrix(g: Geometry) -> np.ndarray:
    """Dense (N*M, n*n) matrix of R_h from scalar loops (brute force).

    Row index l*M + k, column index j*n + i.
    """
    n, N, M = g.n, g.n_angles, g.n_bins
    A = np.zeros((N * M, n * n), dtype=np.float64)
    for l in range(N):
        for j in range(n):
            for i in range(n):
                t = g.bin_coordinate_scalar(i, j, l)
                k = math.floor(t)
                a = t - k
                col = j * n + i
                if 0 <= k < M:
                    A[l * M + k, col] += 1.0 - a
                if 0 <= k + 1 < M:
                    A[l * M + k + 1, col] += a
    return A


def radon_adj_at(g: Geometry, v: np.ndarray, pixels) -> np.ndarray:
    """(R_h^* v)[j, i] for a list of (j, i) pixels only, with scalar geometry
    (for spot checks of full-size backprojections)."""
    v = np.asarray(v, dtype=np.float64)
    out = np.zeros(len(pixels))
    for q, (j, i) in enumerate(pixels):
        acc = 0.0
        for l in range(g.n_angles):
            t = g.bin_coordinate_scalar(i, j, l)
            k = math.floor(t)
            a = t - k
            if 0 <= k < g.n_bins:
                acc += (1.0 - a) * v[l, k]
            if 0 <= k + 1 < g.n_bins:
                acc += a * v[l, k + 1]
        out[q] = acc
    return out


def radon_fwd_at(g: Geometry, u: np.ndarray, bins) -> np.ndarray:
    """(R_h u)[l, k] for a list of (l, k) bins only: the pixels with
    floor(t) = k contribute (1 - alpha) u, those with floor(t) = k - 1
    contribute alpha u (for spot checks of full-size projections)."""
    u = np.asarray(u, dtype=np.float64)
    out = np.zeros(len(bins))
    cache = {}
    for q, (l, k) in enumerate(bins):
        if l not in cache:
            t = g.bin_coordinate(l)
            kk = np.floor(t)
            cache = {l: (kk.astype(np.int64), t - kk)}
        kk, a = cache[l]
        out[q] = np.sum(((1.0 - a) * u)[kk == k]) + np.sum((a * u)[kk == k - 1])
    return out
