"""CPU oracle for ML(n)BiCGStab (test infrastructure only).

A plain, slow, fp64 / complex128 implementation of what the GPU library
computes, written from the paper (Yeung, "An introduction to ML(n)BiCGStab",
arXiv 1106.3678).  Only the tests, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import it; the GPU library never
does, and the two share no code.

Modules:
  index      -- the index functions g_n, r_n (Section 2, Table 2.1)
  mlbicgstabt-- ML(n)BiCGStabt: Algorithm 4.1 as one loop over k, with the
                preconditioner of Algorithm 7.1 and the omega guard of
                eq. (5.1); M = I unless given
  mlbicg     -- ML(n)BiCG, Algorithm 3.1 (only used to pin the oracle)
  ilu0       -- ILU(0), point and 3x3-block, and the (M^{-1}, M^{-H}) pair built
                from it (the preconditioner of the paper's experiments, Section 5)

Parity status: every function is pinned by a CPU test (Table 2.1, n=1 equals
BiCGStab, n=1 with the kappa guard equals the guarded BiCGStab of Sleijpen and
van der Vorst, the preconditioned iteration equals the iteration on A M^{-1}
(Section 4.3), finite termination against LU, FOM/GMRES relations,
Algorithm 3.1 and eq. (4.1), Table 4.3 operation counts; ILU(0) by its defining
identity (L U = A on A's pattern), exact LU without fill, and an elimination in
another loop order) except the paper's
sample execution (Section 7), which prints no outputs: parity unpinned for
that case only.
"""
from .index import g_n, r_n
from .mlbicgstabt import OpCounter, Result, mlbicgstabt, true_error
from .mlbicg import mlbicg
from .ilu0 import ilu0, ilu0_bsr3, ilu0_precond

__all__ = ["g_n", "r_n", "OpCounter", "Result", "mlbicgstabt", "true_error", "mlbicg", "ilu0", "ilu0_bsr3",
           "ilu0_precond"]
