"""FP64 CPU oracle of the optimisation-suggestion method.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU-baseline
leg of the benchmark may import or run anything in this package; the product
path never does, and it shares no code with the GPU implementation (the only
common dependency is the seeded input generator, which holds none of the
method's arithmetic).

It is written for a reader holding the paper: every function names the passage
it follows, steps run in the paper's order, and library routines (a Cholesky
factorisation, a triangular solve, a sort) are the only building blocks.

Modules
  plain      Tiers 1-3 (Section 2): cycle-normalised features, per-optimisation
             ridge regression trained on before/after pairs (Sections 2, 3.4, 5),
             subset composition, threshold + top-n ranking.
  surrogate  The learned MLP that predicts a whole subset table (an extension
             beyond the paper), its hand-written backward and Adam.
  checks     Tolerance-aware comparison of suggestion lists.
"""
