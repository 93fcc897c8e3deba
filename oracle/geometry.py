"""Discretization geometry (thesis §3.1, "Discretization").

Readings taken here (the thesis text is 1-based and partly garbled):
* Pixel centres (§3.1, grid G_h): with 0-based i, j in [0, n),
  x_i = h (i - (n-1)/2) and y_j = h (j - (n-1)/2), the same points as the
  thesis' h (i - (n+1)/2) for 1-based i.  Images are stored u[j, i]
  (row j = y index, column i = x index).  The grid is square (n = m).
* Angles: theta_l = pi l / N, l in [0, N), uniform on [0, pi), unless explicit
  angles are given (§3.1 allows arbitrary theta_1, ..., theta_N).
* Detector bins (§3.1, bin spacing Delta s, rotation centre between the two
  middle bins for even M): 0-based bin k has centre s_k = ds (k - (M-1)/2).
* Bin coordinate (§3.1, definition of R_h^*): a pixel at (x, y) projects to
  s = x cos(theta) + y sin(theta); its continuous bin coordinate is
  t = s / ds + (M-1)/2, so that t = k exactly at bin centre k.  The pixel lies
  between bins floor(t) and floor(t)+1.  (The printed index formula carries a
  stray half-integer offset; this is the reading that places bin centres as
  the text describes, and it holds for odd M as well.)
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass(frozen=True)
class Geometry:
    """Square n x n image, N parallel-beam angles, M detector bins."""
    n: int
    n_angles: int
    n_bins: int
    h: float = 1.0
    ds: float = 1.0
    thetas: tuple | None = None   # explicit angles theta_1..theta_N (the thesis allows any)

    def theta(self, l: int) -> float:
        return float(self.thetas[l]) if self.thetas is not None else math.pi * l / self.n_angles

    def angles(self) -> np.ndarray:
        """theta_l = pi * l / N for l in [0, N), or the explicit angles."""
        if self.thetas is not None:
            return np.asarray(self.thetas, dtype=np.float64)
        return math.pi * np.arange(self.n_angles, dtype=np.float64) / self.n_angles

    def pixel_centres(self) -> np.ndarray:
        """x_i = h (i - (n-1)/2), also the y_j values (§3.1, grid G_h)."""
        return self.h * (np.arange(self.n, dtype=np.float64) - (self.n - 1) / 2.0)

    def bin_centres(self) -> np.ndarray:
        """s_k = ds (k - (M-1)/2)."""
        return self.ds * (np.arange(self.n_bins, dtype=np.float64) - (self.n_bins - 1) / 2.0)

    def bin_coordinate(self, l: int) -> np.ndarray:
        """t[j, i] = (x_i cos theta_l + y_j sin theta_l)/ds + (M-1)/2 for angle l."""
        th = self.theta(l)
        x = self.pixel_centres()
        s = x[None, :] * math.cos(th) + x[:, None] * math.sin(th)
        return s / self.ds + (self.n_bins - 1) / 2.0

    def bin_coordinate_scalar(self, i: int, j: int, l: int) -> float:
        """The same quantity for one pixel, with scalar math only."""
        th = self.theta(l)
        x = self.h * (i - (self.n - 1) / 2.0)
        y = self.h * (j - (self.n - 1) / 2.0)
        return (x * math.cos(th) + y * math.sin(th)) / self.ds + (self.n_bins - 1) / 2.0
