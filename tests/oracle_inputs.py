"""Test-side assembly of problem inputs from the seeded generator (synth) and
the FP64 oracle's projector: u0, the metal trace D0 and the bounds C, rounded
to FP32 once and handed to both the oracle and the GPU path."""
from __future__ import annotations

import numpy as np

import synth
from oracle import geometry, pdrq, radon


def f32(x):
    return np.asarray(x, dtype=np.float32).astype(np.float64)


def build(w: synth.Workload):
    """(geometry, u0, mask, bound) in float64 holding float32-representable values.

    u0 = R_h P + p max(R_h P_tissue) z; D0 = {R_h 1_metal > 0};
    C = 0.95 R_h P_tissue on D0 (zero elsewhere).
    """
    g = geometry.Geometry(w.n, w.n_angles, w.n_bins)
    tissue_proj = radon.radon_fwd(g, w.tissue)
    clean = radon.radon_fwd(g, w.phantom)
    sigma_n = w.noise_level * float(tissue_proj.max())
    u0 = clean + sigma_n * w.noise
    mask = radon.radon_fwd(g, w.metal.astype(np.float64)) > 0
    bound = np.where(mask, 0.95 * tissue_proj, 0.0)
    return g, f32(u0), mask, f32(bound)


def oracle_problem(g, u0, mask, bound, lam):
    return pdrq.Problem(g, u0, mask, bound, lam)


def random_state(n: int, N: int, M: int, seed: int, vb2_scale: float, u_scale: float = 1.0):
    """A seeded iterate (u, vb1, vb2) for one-step parity checks, float64
    holding float32-representable values: u ~ u_scale U[0, 1), vb1 ~ 0.01 N(0, 1),
    vb2 ~ vb2_scale N(0, 1) (callers pass lambda~/tau, the dual ball's radius).
    A small u_scale keeps the projection of u below the bounds on the metal
    trace, so that its constraints are active."""
    rng = np.random.default_rng(seed)
    u = f32(u_scale * rng.uniform(0.0, 1.0, (n, n)))
    vb1 = f32(0.01 * rng.standard_normal((N, M)))
    vb2 = f32(vb2_scale * rng.standard_normal((2, n, n)))
    return u, vb1, vb2


def random_problem(N: int, M: int, seed: int, trace_fraction: float = 0.03):
    """Seeded problem data for one-step checks at sizes where projecting a
    phantom on the host would take too long: u0 = 50 |z| (the scale of a
    projection of unit densities over tens of pixels), a metal-trace mask of
    about trace_fraction of the bins, and bounds C = 0.9 u0 on it.  Returns
    (u0, mask, bound) in float64 holding float32-representable values."""
    rng = np.random.default_rng(seed)
    u0 = f32(50.0 * np.abs(rng.standard_normal((N, M))))
    mask = rng.uniform(0.0, 1.0, (N, M)) < trace_fraction
    bound = f32(np.where(mask, 0.9 * u0, 0.0))
    return u0, mask, bound
