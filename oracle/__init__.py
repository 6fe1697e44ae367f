"""CPU float64 oracle for M-IHS ridge regression.

TEST INFRASTRUCTURE ONLY: tests, the package's smoke check and the benchmark's
CPU-baseline leg may import this package; the product path (the HIP library
and its Python binding) never does, and shares no code with it.

Modules:
  hashes    - MurmurHash3_x86_32 and Philox-4x32-10 with Box-Muller, from their
              published definitions (the sketch's random source)
  sketches  - Gaussian, SRHT and CountSketch sketches (Lemma 3)
  solver    - closed forms, momentum (Theorem 1, Corollary 4), CG and
              AAb_Solver (Algorithm 6) inner solvers, M-IHS (Algorithm 1),
              dense ridge backward
"""
from . import hashes, sketches, solver  # noqa: F401
