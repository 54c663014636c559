"""FP64 CPU oracle for the multigrid pressure-projection solve.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this package; the solver library never does, and the
two share no code.  It is plain and slow on purpose: numpy/scipy, FP64 (FP32 only
where it emulates the single-precision inner cycles), written so that each step can
be checked against the paper by eye.

  operator   - face coefficients, the finite-volume operator A, invariants helpers
  multigrid  - red-black Gauss-Seidel, transfers, coarsening, V-cycle, solves
  exact      - bordered dense / sparse direct solves, FFT + Thomas for z-only fields
  adjoint    - adjoint solve and the face / density gradients
  projection - the Runge-Kutta stage around the solve: source and velocity projection
  cutcell    - fractional-area cut cells from a body level set, small-cell merging

Parity status: every function is pinned by a CPU test against something other
than itself (closed-form eigenfunctions, brute-force dense algebra, library
pseudo-inverse, independent direct solvers, identities).  The convergence *rate*
of the V-cycle has no published value to pin it to: the paper states only that the
method does not slow down as the grid grows past ten million cells.
"""
from . import adjoint, cutcell, exact, multigrid, operator, projection  # noqa: F401
from .multigrid import Hierarchy, setup, solve, solve_mixed, vcycle  # noqa: F401
from .operator import Level, apply, face_coeffs_from_rho, project  # noqa: F401
