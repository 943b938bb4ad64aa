"""CPU oracle for RACE-scheduled SymmSpMV -- TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously-correct reference implementations written from the
paper (Alappat et al., "A Recursive Algebraic Coloring Technique for
Hardware-Efficient Symmetric Sparse Matrix-Vector Multiplication"):

* ``symmspmv``  -- the product y = A x from the upper-triangle CRS storage
  (Algorithm "SymmSpMV", Section 3.2) and its plain definitions.
* ``schedule``  -- the RACE schedule: BFS levels (Algorithm "Construction of
  levels", Eq. (level), Section 4.1), level permutation, distance-2 level
  groups (Section 4.2), load balancing (Algorithm "Load Balancing",
  Section 4.3), recursion with the epsilon level aggregation
  (Section 4.4) and the effective row count / parallel efficiency
  (Section 5).
* ``checker``   -- brute-force conflict checker for a schedule; shares no
  code with ``schedule``.
* ``perfmodel`` -- the roofline intensities of Section 3 (Eqs. SpMV and
  SymmSpMV intensity).
* ``mlp``       -- float64 forward/backward of the small cost-model network.
* ``gauss_seidel`` -- Gauss-Seidel sweeps over a row order (distance-1
  schedules), and the order a schedule runs its rows in.
* ``kaczmarz``  -- Kaczmarz sweeps (row projections) over a row order
  (distance-2 schedules).
* ``powers``    -- matrix powers and polynomials built from products.

Only the tests, the smoke entry and the benchmark's CPU-baseline leg may
import this package.  The product path never calls it.
"""
