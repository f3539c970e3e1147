"""CPU FP64 oracle for the regional multigrid preconditioned CG method.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import or call
this package: only the tests, the smoke check and the CPU-baseline leg of the
benchmark use it.  It shares no code with the HIP library.

The oracle computes the method two independent ways (paper, Sections 3.1-3.6):

* ``regional``  -- the regional algorithm written out: region boxes and the
  boolean map Psi as index operations, per-region stencils, the per-region
  Galerkin product, interface sums Psi^T Psi, the regional restriction
  formula, Chebyshev smoothing, a dense coarse solve, and CG.
* ``composite`` -- plain composite multigrid with sparse matrices
  (A, P, R = P^T, RAP), the textbook structure the regional form must equal
  (Lemma on Psi [[A]] Psi^T = A, Lemmas on P and R, Galerkin theorem).

Readings of points the paper leaves open are listed in each module.
Functions whose result has no independent check say "parity unpinned".
"""
