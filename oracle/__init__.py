"""FP64 CPU oracle for the arrowhead KKT solve of the structure-exploiting
interior point method (Kardos, Kourounis, Schenk, arXiv 1907.05420).

TEST INFRASTRUCTURE ONLY. Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this package. The GPU library shares no code with
it and never calls it.

Contents
  arrowhead  -- the monolithic KKT matrix of Eq. hessianPerm with the MPOPF
                border of Eq. B12N (plain assembly, scipy.sparse).
  ldlt       -- plain dense LDL^T with 1x1 pivots in the given order, a static
                sign-preserving pivot perturbation, inertia by Sylvester's law.
  schur      -- Algorithm 1 (Schur-complement decomposition, Eqs. SCform,
                SCsolve, SCsolve1), the MPOPF local-Schur blocks of Eqs.
                LocalSchurBs / LocalSchurBs3, the monolithic reference solve and
                FP64 iterative refinement.

Every result the method produces here has a plain definition: x solves K x = b
for the nonsingular K, S is the Schur complement of the block diagonal, and the
inertia is the sign count of K's eigenvalues. Pins (tests marked "not gpu")
check these against numpy/LAPACK brute force, eigvalsh and the paper's
structural identities.

Parity status: the mixed-precision refinement has no pin of its own beyond
the FP64 oracle solution (parity unpinned by the paper for that mode).
"""
