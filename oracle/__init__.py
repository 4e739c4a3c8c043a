"""The oracle: a plain, slow, CPU-only float64 implementation of what the
Chebyshev sparse-matrix-function path computes.

TEST INFRASTRUCTURE.  Only the tests, the smoke check and the CPU-baseline leg
of the benchmark may import or execute anything in this package; the product
(the HIP library and its Python binding) never does, and the two share no code.

  chebyshev.py  scalar formulas: Eq. 5 coefficients, Eq. 7 degree, Eqs. 9/11
                occupations, Eq. 6 penalty, mu bisection, eigenvalue extraction
  csr_chain.c   the truncated recursion of Eq. 4 and the sums of Eq. 1 in
                plain scalar CSR (compiled with gcc)
  csr.py        ctypes access to csr_chain.c, block <-> scalar CSR conversion
  pipeline.py   the method in the paper's order (FOE, matrix powers, eigenvalues)
  dense.py      exact dense definitions (generalized eigendecomposition) and the
                error measures of Eqs. 12 and 13

Pins: every function above is checked by tests/test_oracle_*.py against
closed forms, library routines, invariants or brute force (see those files).
"""
