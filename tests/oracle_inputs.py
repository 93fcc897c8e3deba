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
