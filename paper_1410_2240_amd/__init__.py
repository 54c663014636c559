"""MI355X-native multigrid pressure-projection solve (HIP kernels behind a C ABI).

The solver library (libmgpoisson.so, built in-tree by `python -m
paper_1410_2240_amd.build`) does all the work; this package only marshals
arguments.  See include/mg.h for the ABI.
"""
from .solver import MG, MGError, coeffs_from_rho, workspace_size  # noqa: F401
from .autograd import PoissonSolve, poisson_solve  # noqa: F401
from . import cutcell  # noqa: F401
