"""Discrete gradient, divergence and TV (thesis §3.1, "Discretization").

nabla_h: forward differences with Neumann boundary, zero in the last column
(x direction, index i) and the last row (y direction, index j).
div_h = -nabla_h^T: backward differences with Dirichlet boundary, as the
piecewise formula of §3.1 gives (first entry p[0], interior p[i] - p[i-1],
last entry -p[n-2]).
TV: the isotropic one-norm sum_{i,j} sqrt(q1^2 + q2^2) of §3.1 (the thesis'
"max norm" ball of its resolvent is read as the pointwise Euclidean ball,
which is the dual of this norm).

Layout: u[j, i]; a gradient field p has shape (2, n, n) with p[0] the x
(column) difference and p[1] the y (row) difference.
"""
from __future__ import annotations

import numpy as np


def grad(u: np.ndarray, h: float = 1.0) -> np.ndarray:
    """nabla_h u = (d_x u, d_y u), forward differences, zero on the far edge."""
    u = np.asarray(u, dtype=np.float64)
    p = np.zeros((2,) + u.shape, dtype=np.float64)
    p[0, :, :-1] = (u[:, 1:] - u[:, :-1]) / h
    p[1, :-1, :] = (u[1:, :] - u[:-1, :]) / h
    return p


def div(p: np.ndarray, h: float = 1.0) -> np.ndarray:
    """div_h p = (d_1(p) + d_2(p)) / h with the piecewise backward differences
    of §3.1, so that <nabla_h u, p> = <u, -div_h p>."""
    p = np.asarray(p, dtype=np.float64)
    p1, p2 = p[0], p[1]
    n_r, n_c = p1.shape
    d1 = np.zeros_like(p1)
    d1[:, 0] = p1[:, 0]
    d1[:, 1:n_c - 1] = p1[:, 1:n_c - 1] - p1[:, 0:n_c - 2]
    d1[:, n_c - 1] = -p1[:, n_c - 2]
    d2 = np.zeros_like(p2)
    d2[0, :] = p2[0, :]
    d2[1:n_r - 1, :] = p2[1:n_r - 1, :] - p2[0:n_r - 2, :]
    d2[n_r - 1, :] = -p2[n_r - 2, :]
    return (d1 + d2) / h


def tv(u: np.ndarray, h: float = 1.0) -> float:
    """||nabla_h u||_1 = sum sqrt((d_x u)^2 + (d_y u)^2)  (§3.1)."""
    p = grad(u, h)
    return float(np.sum(np.sqrt(p[0] ** 2 + p[1] ** 2)))
