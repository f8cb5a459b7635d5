"""MI355X-native PCG with an AINV approximate-inverse preconditioner for the
five-point elliptic sea-surface equation (Cuomo, De Michele, Farina,
Chinnici; Algorithm 1 with P = Z D^-1 Z^T).

The compute path is libpcgainv.so (hand-written HIP for gfx950 behind a C
ABI declared in include/pcgainv.h); this package only marshals arguments.
"""
from .api import (AInv, Batch, CsrMatrix, HwStream, SolveResult, Solver, Stencil5, ainv_setup,  # noqa: F401
                  workspace_size, fsai_band_setup, pcg_solve, pcg_solve_mixed)
from ._lib import PcgaError  # noqa: F401
