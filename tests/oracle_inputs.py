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


def random_state(n: int, N: int, M: int, seed: int, vb2_scale: float):
    """A seeded iterate (u, vb1, vb2) for one-step parity checks, float64
    holding float32-representable values: u ~ U[0, 1), vb1 ~ 0.01 N(0, 1),
    vb2 ~ vb2_scale N(0, 1) (callers pass lambda~/tau, the dual ball's radius)."""
    rng = np.random.default_rng(seed)
    u = f32(rng.uniform(0.0, 1.0, (n, n)))
    vb1 = f32(0.01 * rng.standard_normal((N, M)))
    vb2 = f32(vb2_scale * rng.standard_normal((2, n, n)))
    return u, vb1, vb2
