"""FP64 CPU oracle of the trace-minimization eigensolver.

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow, obviously correct
reference that the GPU library is checked against.  It is imported by the test
suite, by the smoke check and by the CPU-baseline leg of the benchmark, never by
the GPU package, and it shares no code with it (the only common input is the
seeded problem generator in ``workloads``).

Contents (each function cites the passage of Tsuchida & Choe, "Iterative
diagonalization of symmetric matrices in mixed precision", that it follows):

* ``tracemin``  -- energy and gradient (Fig. 2, Algorithm-1 and -2), Cholesky
  orthonormalization (Fig. 4), the nonlinear-CG driver (Fig. 1, Eq. 8), the
  diagonal preconditioner (Eq. 18), the final Rayleigh-Ritz step (Eq. 9) and a
  brute-force dense eigensolve for tiny N.
* the generalized problem H x = lambda S x with S symmetric positive definite
  (Sec. 2.1): energy and gradient in the S metric, S-orthonormalization, and
  the same driver with ``solve(..., S=S)``.
* ``jacobi.c``  -- cyclic Jacobi eigensolver in plain C, built by ``build.py``.

Parity pins: see ``tests/test_oracle_*.py``.  The only routine without an
independent pin is noted in its docstring.
"""

from .tracemin import (  # noqa: F401
    csr_matrix,
    spmm,
    energy_gradient_alg1,
    energy_gradient_alg2,
    cholesky_upper,
    upper_triangular_inverse,
    orthonormalize,
    jacobi_eigh,
    rayleigh_ritz,
    jacobi_preconditioner,
    gershgorin_bounds,
    chebyshev_preconditioner,
    line_step,
    solve,
    brute_force_lowest,
    energy_gradient_generalized,
    orthonormalize_generalized,
    brute_force_generalized,
    OracleOptions,
    OracleResult,
)
