"""FP64 CPU oracle for preconditioned primal-dual TV/metal CT reconstruction.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously correct
NumPy implementation of what the GPU path computes, written from
C. Schiffer, "TV-regularized CT reconstruction and metal artifact reduction
using inequality constraints with preconditioning" (2018, arXiv:1810.03275).
Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import or run it; the product library never does.  It shares no code, table or
constant with the GPU path; the only common module is the seeded input
generator, which holds none of the method's arithmetic.

Modules (each function cites the thesis passage it follows):
  geometry  pixel grid, angles, detector bins, bin coordinate     (§3.1)
  radon     R_h^* (pixel-driven interpolation) and R_h (its transpose)  (§3.1)
  tv        forward-difference gradient, divergence, isotropic TV  (§3.1)
  precond   periodic-Laplacian symbol, inverse-norm preconditioner (§4.3, §4.3.1, §4.4)
  prox      pointwise resolvents                                   (§3.3, §4.4, §3.5, §4.5)
  power     power iterations for ||R_h|| and the constant c       (§4.3, §4.3.1, §5.1)
  pdrq      problem setup, normalization, Algorithm PDRQS1         (§4.4, §5.1)
  cp        Algorithm CP (Chambolle-Pock) as an independent solver (§3.4)
  gap       FP64 primal/dual record (a reading; the thesis defines none)
  d0        metal-trace estimate: threshold, dilate, project        (results, real metal)
  admm      ADMM with inner PCG and isotropic soft thresholding     (§4.6)
  pdrq3     the PDRQ3 splitting (fit in the dual's quadratic part)  (§4.4)
  parallel  R_h / R_h^* split over angle blocks in worker processes (§3.1)

Readings of passages that are silent, ambiguous or garbled are listed in the
header of the module that takes them and collected in the repository's design
notes.  Parity status: every function is pinned by the tests under tests/
(test_oracle_*.py) except where its docstring says "parity unpinned".
"""
from . import geometry, radon, tv, precond, prox, power, pdrq, cp, gap, d0, admm, pdrq3  # noqa: F401

__all__ = ["geometry", "radon", "tv", "precond", "prox", "power", "pdrq", "cp", "gap", "d0", "admm", "pdrq3"]
