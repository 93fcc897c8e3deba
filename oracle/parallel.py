"""The oracle's R_h and R_h^* (§3.1) split over blocks of angles that worker
processes project.

Each block is a sub-geometry holding the same angle values, so every bin of
R_h is the oracle's own sum (radon.radon_fwd on the block) and R_h^* adds the
blocks' partial images in block order.  Only the order in which the per-angle
contributions to a pixel are added differs from the serial oracle (FP64, so
the results agree to rounding, ~1e-15 relative).  Used to run the oracle on
more host cores: the stored full-size values and the timed host baseline.
"""
from __future__ import annotations

from concurrent.futures import ProcessPoolExecutor

import numpy as np

from . import radon
from .geometry import Geometry


class AngleBlocks:
    """fwd(u) = R_h u and adj(v) = R_h^* v of geometry g on `workers`
    processes (4 blocks per worker)."""

    def __init__(self, g: Geometry, workers: int):
        self.workers = int(workers)
        self.pool = ProcessPoolExecutor(self.workers)
        th = g.angles()
        self.blocks = np.array_split(np.arange(g.n_angles), 4 * self.workers)
        self.subs = [Geometry(g.n, len(b), g.n_bins, g.h, g.ds,
                              thetas=tuple(float(t) for t in th[b])) for b in self.blocks]

    def fwd(self, u):
        return np.concatenate(list(self.pool.map(radon.radon_fwd, self.subs,
                                                 [u] * len(self.subs))), axis=0)

    def adj(self, v):
        out = None
        for part in self.pool.map(radon.radon_adj, self.subs, [v[b] for b in self.blocks]):
            out = part if out is None else out + part
        return out

    def close(self):
        self.pool.shutdown()
