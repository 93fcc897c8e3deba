"""Write the stored expected values of the full-size parity tests.

Every value written here comes from the FP64 oracle (oracle/) on inputs from
the seeded generator (synth) assembled by tests/oracle_inputs.py; nothing is
read from the GPU path.  Run from the repository root:

  python tests/golden/make_golden.py c2    # ~25 min, one core
  python tests/golden/make_golden.py c5    # ~35 min, one core

c2: the 512^2 x 720 x 768 workload with 2 metal discs (alpha = 0.005), set up
    by the oracle's power iterations from the workload's start images (§5.1,
    §4.3.1), then 500 PDRQS1 iterations (§4.4) from the zero state.  Stored:
    beta, c, lambda~, the image after 500 iterations (float32) and the gap
    records after every 100th iteration.
c5: the 2048^2 x 2880 x 3072 geometry with 4 metal discs; one PDRQS1 step
    from a seeded random iterate with fixed step constants beta = 2430,
    c = 1.25 (beta is close to ||R_h|| ~ sqrt(N n) for this geometry; any
    positive constants define the same test).  A full oracle step at this
    size takes three projector passes of ~11 min each, so only sampled
    entries are stored: u_new at sampled pixels, vb1 at sampled bins, vb2 at
    sampled pixels of both planes, and the L2 norms of the three arrays.
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(HERE))

import synth  # noqa: E402
from oracle import pdrq  # noqa: E402
from oracle_inputs import build, f32, random_state  # noqa: E402

C5_BETA = 2430.0
C5_C = 1.25
C5_STATE_SEED = 5005
C5_SAMPLE_SEED = 5006


def c5_samples(n: int, N: int, M: int):
    """Sampled pixel and bin indices of the 2048^2 one-step check: random
    ones plus the corners, the centre and the detector ends."""
    rng = np.random.default_rng(C5_SAMPLE_SEED)
    pix = rng.integers(0, n, (2000, 2))
    pix = np.concatenate([pix, [[0, 0], [0, n - 1], [n - 1, 0], [n - 1, n - 1],
                                [n // 2, n // 2], [n // 2 - 1, n // 2]]])
    bins = np.stack([rng.integers(0, N, 2000), rng.integers(0, M, 2000)], axis=1)
    bins = np.concatenate([bins, [[0, 0], [0, M - 1], [N - 1, 0], [N - 1, M - 1],
                                  [N // 2, M // 2], [N // 4, M // 2]]])
    return pix.astype(np.int64), bins.astype(np.int64)


def make_c2(path: str) -> None:
    w = synth.workload("C2")
    g, u0, mask, bound = build(w)
    t0 = time.time()
    s = pdrq.setup(pdrq.Problem(g, u0, mask, bound, w.alpha), pdrq.Params(),
                   f32(w.start_norm), f32(w.start_precond))
    print(f"c2 setup: beta {s.beta:.9g} c {s.c:.9g} ({time.time() - t0:.0f} s)", flush=True)
    st = pdrq.zero_state(s)
    records = []
    for k in range(w.iters):
        if (k + 1) % 100 == 0:
            from oracle import gap
            prev = st.u
            st, y1, wd = pdrq.step(s, st, return_dual=True)
            records.append(gap.record(s, st.u, y1, wd, prev))
            print(f"c2 iteration {k + 1} ({time.time() - t0:.0f} s) record {records[-1]}",
                  flush=True)
        else:
            st = pdrq.step(s, st)
    np.savez_compressed(path, u=st.u.astype(np.float32), beta=s.beta, c=s.c, lam_t=s.lam_t,
                        iters=w.iters, records=np.array(records),
                        record_iters=np.arange(100, w.iters + 1, 100))
    print("wrote", path, flush=True)


def make_c5(path: str) -> None:
    w = synth.workload("C5")
    g, u0, mask, bound = build(w)
    n, N, M = g.n, g.n_angles, g.n_bins
    print("c5 inputs built", flush=True)
    t0 = time.time()
    s = pdrq.setup(pdrq.Problem(g, u0, mask, bound, w.alpha), pdrq.Params(),
                   beta=C5_BETA, c=C5_C)
    u, vb1, vb2 = random_state(n, N, M, C5_STATE_SEED, s.lam_t / s.params.tau)
    st = pdrq.state_from(s, u, vb1, vb2)
    print(f"c5 state caches ({time.time() - t0:.0f} s)", flush=True)
    new = pdrq.step(s, st)
    print(f"c5 step ({time.time() - t0:.0f} s)", flush=True)
    pix, bins = c5_samples(n, N, M)
    np.savez_compressed(
        path, beta=C5_BETA, c=C5_C, pix=pix, bins=bins,
        u=new.u[pix[:, 0], pix[:, 1]], vb1=new.vb1[bins[:, 0], bins[:, 1]],
        vb2_0=new.vb2[0][pix[:, 0], pix[:, 1]], vb2_1=new.vb2[1][pix[:, 0], pix[:, 1]],
        norms=np.array([np.linalg.norm(new.u), np.linalg.norm(new.vb1),
                        np.linalg.norm(new.vb2)]))
    print("wrote", path, flush=True)


if __name__ == "__main__":
    which = sys.argv[1] if len(sys.argv) > 1 else "c2"
    if which == "c2":
        make_c2(os.path.join(HERE, "c2_pdrqs1_500.npz"))
    elif which == "c5":
        make_c5(os.path.join(HERE, "c5_step_sampled.npz"))
    else:
        raise SystemExit("usage: make_golden.py c2|c5")
