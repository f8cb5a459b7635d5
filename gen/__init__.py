"""Seeded synthetic inputs shared by the oracle side and the device side.

This package only builds *inputs*: the coefficients of the 5-point elliptic
operator (eq. (8) coefficients placed as in the five-point system eq. (10)),
land masks, bathymetry and right-hand sides, and general sparse SPD matrices
of unstructured point clouds in CSR (`unstructured`).  It holds none of the
solver's arithmetic (no PCG, no approximate inverse).
"""
from .orca import (  # noqa: F401
    Problem,
    box_problem,
    orca_problem,
    ensemble_problems,
    rhs_normal,
    CONFIG_SEED_BASE,
)
from .unstructured import CsrProblem, csr_from_grid, unstructured_problem  # noqa: F401,E402
