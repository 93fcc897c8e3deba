"""Write the stored expected values of the full-size parity tests.

Every value written here comes from the FP64 oracle (oracle/) on inputs from
the seeded generator (synth) assembled by tests/oracle_inputs.py; nothing is
read from the GPU path.  Run from the repository root:

  GOLDEN_WORKERS=4 python tests/golden/make_golden.py c2   # ~100 core-minutes
  GOLDEN_WORKERS=2 python tests/golden/make_golden.py c5   # ~40 core-minutes
  python tests/golden/make_golden.py c3                    # ~15 min, one core
  GOLDEN_WORKERS=7 python tests/golden/make_golden.py c5run  # ~2 hours

GOLDEN_WORKERS > 1 splits the oracle's projector over angle blocks in that
many worker processes.

c2: the 512^2 x 720 x 768 workload with 2 metal discs (alpha = 0.005), set up
    by the oracle's power iterations from the workload's start images (§5.1,
    §4.3.1), then 500 PDRQS1 iterations (§4.4) from the zero state.  Stored:
    beta, c, lambda~, the image after 500 iterations (float32), the gap
    records after every 100th iteration and, with each record, ||y1||, ||wg||
    (wg = y1 + b off the metal trace, C~ on it: G*'s first-order change is
    <dy1, wg>) and ||u||.
c5: the 2048^2 x 2880 x 3072 geometry; one PDRQS1 step from a seeded
    random iterate (image scale STEP_U_SCALE), on seeded problem data (tests/oracle_inputs.py
    random_problem: projecting a phantom on the host would take three more
    projector passes), lambda = 0.005, with fixed step constants beta = 2430,
    c = 1.25 (beta is close to ||R_h|| ~ sqrt(N n) for this geometry; any
    positive constants define the same test).  A full oracle step at this
    size takes three projector passes of ~11 min each, so only sampled
    entries are stored: u_new at sampled pixels, vb1 at sampled bins, vb2 at
    sampled pixels of both planes, and the L2 norms of the three arrays.
c5run: the 2048^2 geometry on the same kind of seeded problem data, beta and c
    fixed as for c5, 20 PDRQS1 iterations from the zero state; the image at
    sampled pixels, vb1 at sampled bins and the three arrays' norms.
c3: the five image sizes of the uneven batch (n in {256, 384, 512, 768,
    1024}, N = round(1.4 n), M = 1.5 n); per size, two problems on seeded
    problem data and seeded iterates, one PDRQS1 step each with beta =
    sqrt(N n), c = 1.25; sampled entries as for c5.
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
from oracle import geometry  # noqa: E402
from oracle.parallel import AngleBlocks  # noqa: E402
from oracle_inputs import build, f32, random_problem, random_state  # noqa: E402

C5_BETA = 2430.0
C5_C = 1.25
C5_STATE_SEED = 5005
C5_SAMPLE_SEED = 5006
C5_PROBLEM_SEED = 5007
C5_LAMBDA = 0.005
# scale of the seeded iterate's image: small enough that its projection lies
# below the bounds on the metal trace (active constraints), and smooth enough
# in sum that one step does not cancel most of a white-noise image (which
# would leave nabla u_new, and so vb2, dominated by FP32 rounding)
STEP_U_SCALE = 0.02
C3_SIZES = (256, 384, 512, 768, 1024)
C3_C = 1.25
C3_LAMBDA = 0.005


def workers() -> int:
    return int(os.environ.get("GOLDEN_WORKERS", "1"))


def c3_geometry(n: int):
    return n, int(round(1.4 * n)), int(1.5 * n)


def c3_beta(n: int) -> float:
    N = int(round(1.4 * n))
    return float(np.sqrt(N * n))


def c3_seeds(n: int, b: int):
    """(problem seed, state seed, sample seed) of problem b of size n."""
    return 3_000_000 + 10 * n + b, 3_100_000 + 10 * n + b, 3_200_000 + 10 * n + b


def c5_samples(n: int, N: int, M: int, seed: int = C5_SAMPLE_SEED, count: int = 2000):
    """Sampled pixel and bin indices of a one-step check: random ones plus
    the corners, the centre and the detector ends."""
    rng = np.random.default_rng(seed)
    pix = rng.integers(0, n, (count, 2))
    pix = np.concatenate([pix, [[0, 0], [0, n - 1], [n - 1, 0], [n - 1, n - 1],
                                [n // 2, n // 2], [n // 2 - 1, n // 2]]])
    bins = np.stack([rng.integers(0, N, count), rng.integers(0, M, count)], axis=1)
    bins = np.concatenate([bins, [[0, 0], [0, M - 1], [N - 1, 0], [N - 1, M - 1],
                                  [N // 2, M // 2], [N // 4, M // 2]]])
    return pix.astype(np.int64), bins.astype(np.int64)


def make_c2(path: str) -> None:
    w = synth.workload("C2")
    g, u0, mask, bound = build(w)
    t0 = time.time()
    kw = {}
    if workers() > 1:
        ab = AngleBlocks(g, workers())
        kw = dict(fwd=ab.fwd, adj=ab.adj)
    s = pdrq.setup(pdrq.Problem(g, u0, mask, bound, w.alpha), pdrq.Params(),
                   f32(w.start_norm), f32(w.start_precond), **kw)
    print(f"c2 setup: beta {s.beta:.9g} c {s.c:.9g} ({time.time() - t0:.0f} s)", flush=True)
    st = pdrq.zero_state(s)
    records, scales = [], []
    for k in range(w.iters):
        if (k + 1) % 100 == 0:
            from oracle import gap
            prev = st.u
            st, y1, wd = pdrq.step(s, st, return_dual=True)
            records.append(gap.record(s, st.u, y1, wd, prev))
            # sizes that bound how much G* moves with the dual iterate: its
            # first-order change is <dy1, wg>, wg = y1 + b off the trace and C~ on it
            mask = s.problem.mask
            wg = np.where(mask, s.cb, y1 + s.b)
            scales.append([np.linalg.norm(y1), np.linalg.norm(wg), np.linalg.norm(st.u)])
            print(f"c2 iteration {k + 1} ({time.time() - t0:.0f} s) record {records[-1]} "
                  f"scales {scales[-1]}", flush=True)
        else:
            st = pdrq.step(s, st)
    np.savez_compressed(path, u=st.u.astype(np.float32), beta=s.beta, c=s.c, lam_t=s.lam_t,
                        iters=w.iters, records=np.array(records),
                        record_scales=np.array(scales),
                        record_iters=np.arange(100, w.iters + 1, 100))
    print("wrote", path, flush=True)


def one_step_sampled(n, N, M, lam, beta, c, problem_seed, state_seed, sample_seed, count):
    """One oracle PDRQS1 step from a seeded iterate on seeded problem data;
    the sampled entries of the new state and its norms."""
    g = geometry.Geometry(n, N, M)
    u0, mask, bound = random_problem(N, M, problem_seed)
    kw = {}
    if workers() > 1:
        ab = AngleBlocks(g, workers())
        kw = dict(fwd=ab.fwd, adj=ab.adj)
    s = pdrq.setup(pdrq.Problem(g, u0, mask, bound, lam), pdrq.Params(), beta=beta, c=c, **kw)
    u, vb1, vb2 = random_state(n, N, M, state_seed, s.lam_t / s.params.tau, STEP_U_SCALE)
    t0 = time.time()
    st = pdrq.state_from(s, u, vb1, vb2)
    new = pdrq.step(s, st)
    print(f"  {n}x{N}x{M} step ({time.time() - t0:.0f} s)", flush=True)
    pix, bins = c5_samples(n, N, M, sample_seed, count)
    return dict(pix=pix, bins=bins, u=new.u[pix[:, 0], pix[:, 1]],
                vb1=new.vb1[bins[:, 0], bins[:, 1]], vb2_0=new.vb2[0][pix[:, 0], pix[:, 1]],
                vb2_1=new.vb2[1][pix[:, 0], pix[:, 1]],
                norms=np.array([np.linalg.norm(new.u), np.linalg.norm(new.vb1),
                                np.linalg.norm(new.vb2)]))


def make_c5(path: str) -> None:
    out = one_step_sampled(2048, 2880, 3072, C5_LAMBDA, C5_BETA, C5_C, C5_PROBLEM_SEED,
                           C5_STATE_SEED, C5_SAMPLE_SEED, 2000)
    np.savez_compressed(path, beta=C5_BETA, c=C5_C, lam=C5_LAMBDA, **out)
    print("wrote", path, flush=True)


C5_RUN_ITERS = 20
C5_RUN_SEED = 5008


def make_c5_run(path: str) -> None:
    """20 PDRQS1 iterations from the zero state on the 2048^2 x 2880 x 3072
    geometry, seeded problem data (the one-step check's kind), beta and c
    fixed as there; the image at sampled pixels and its norm, and the norms of
    vb1 and vb2, after the last iteration."""
    n, N, M = 2048, 2880, 3072
    g = geometry.Geometry(n, N, M)
    u0, mask, bound = random_problem(N, M, C5_PROBLEM_SEED)
    kw = {}
    if workers() > 1:
        ab = AngleBlocks(g, workers())
        kw = dict(fwd=ab.fwd, adj=ab.adj)
    s = pdrq.setup(pdrq.Problem(g, u0, mask, bound, C5_LAMBDA), pdrq.Params(), beta=C5_BETA,
                   c=C5_C, **kw)
    st = pdrq.zero_state(s)
    t0 = time.time()
    for k in range(C5_RUN_ITERS):
        st = pdrq.step(s, st)
        print(f"  iteration {k + 1} ({time.time() - t0:.0f} s)", flush=True)
    pix, bins = c5_samples(n, N, M, C5_RUN_SEED, 2000)
    np.savez_compressed(path, beta=C5_BETA, c=C5_C, lam=C5_LAMBDA, iters=C5_RUN_ITERS, pix=pix,
                        bins=bins, u=st.u[pix[:, 0], pix[:, 1]],
                        vb1=st.vb1[bins[:, 0], bins[:, 1]],
                        norms=np.array([np.linalg.norm(st.u), np.linalg.norm(st.vb1),
                                        np.linalg.norm(st.vb2)]))
    print("wrote", path, flush=True)


def make_c3(path: str) -> None:
    arrays = {}
    for n in C3_SIZES:
        n, N, M = c3_geometry(n)
        for b in range(2):
            ps, ss, qs = c3_seeds(n, b)
            out = one_step_sampled(n, N, M, C3_LAMBDA, c3_beta(n), C3_C, ps, ss, qs, 500)
            for k, v in out.items():
                arrays[f"n{n}_b{b}_{k}"] = v
    np.savez_compressed(path, **arrays)
    print("wrote", path, flush=True)


if __name__ == "__main__":
    which = sys.argv[1] if len(sys.argv) > 1 else "c2"
    if which == "c2":
        make_c2(os.path.join(HERE, "c2_pdrqs1_500.npz"))
    elif which == "c5":
        make_c5(os.path.join(HERE, "c5_step_sampled.npz"))
    elif which == "c3":
        make_c3(os.path.join(HERE, "c3_step_sampled.npz"))
    elif which == "c5run":
        make_c5_run(os.path.join(HERE, "c5_pdrqs1_20_sampled.npz"))
    else:
        raise SystemExit("usage: make_golden.py c2|c5|c3|c5run")
