"""FP64 CPU oracle for sketched Riemannian CCA / FDA.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute anything in this package: only ``tests/``, ``__graft_entry__.smoke``
and the ``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with
the GPU library (no kernels, headers, helpers, constants or generators); its
only common dependency with the GPU side is the seeded data generator in
``synth``, which holds none of the method's arithmetic.

What it computes, each function citing the passage it follows:

* ``direct``  -- the lambda-canonical correlations and weights (Definition
  of regularised CCA, Section 4) and the regularised FDA weights
  (Definition of FDA, Section 5) as plain closed forms: a Cholesky-whitened
  SVD.  The method is Las Vegas: its fixed point is this exact solution,
  whatever sketch, seed or metric it uses (critical-point theorems of
  Sections 4.2 and 5.2 hold for every metric).
* ``sketch``  -- CountSketch (Section 3) and SRHT (Appendix A definition)
  applied by their definitions, and the counter-based hash (SplitMix64,
  Steele, Lea and Flood 2014) that draws their randomness.
* ``stiefel`` -- the preconditioned generalized-Stiefel components of
  Table 1 (metric, projection through the Sylvester equation, QR retraction,
  transport, Riemannian gradient) and the CCA / FDA costs and gradients
  (Eq. costriemannianccaBrockett, Eq. gradCCA, Eq. lda_riemannian).
* ``metrics`` -- constraint residuals, objective errors and the paper's
  weighted sub-optimality measure (Section 6.1).

Everything is FP64 numpy.  Library routines (matmul, Cholesky, triangular
solve, SVD, QR) serve as single steps only.
"""
from . import direct, sketch, stiefel, metrics  # noqa: F401
