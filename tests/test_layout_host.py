"""Host-side sliced-ELL layout (no GPU): the structure the kernels rely on.

A table slice keeps its column-offset table in one wavefront register (lane c
holds step c), so no table slice may have more than 64 entry steps, at any
target width the solver accepts.  The factors of the 182x149 and 362x292
ORCA-shaped grids at drop tolerance 0.01 have one-lane-per-row slices whose
offset union is wider than 64 at target width 64.
"""
import numpy as np
import pytest

import paper_1210_1878_amd as P
from gen import orca


@pytest.mark.parametrize("nx,ny,seed", [(182, 149, orca.CONFIG_SEED_BASE + 1), (362, 292, 5)])
@pytest.mark.parametrize("width", [1, 8, 24, 32, 48, 64])
def test_table_slices_fit_one_register(nx, ny, seed, width):
    p = orca.orca_problem(nx, ny, seed)
    A = P.Stencil5.from_problem(p)
    G = P.ainv_setup(A, 0.01)
    info = G.layout_info(width)
    for m in ("zt", "z"):
        d = info[m]
        assert d["table_width_max"] <= 64
        assert d["entries"] >= G.nnz_off            # every entry stored, with padding
        assert d["entries"] % 64 == 0
        assert d["index_bytes"] == 2                # distances fit 16 bits on these grids
    if width == 64:
        # the cap binds here: some slices fall back to per-lane indices that
        # would otherwise have taken a table wider than one register
        assert info["zt"]["width_max"] == 64


def test_layout_info_rejects_bad_width():
    p = orca.orca_problem(37, 23, 5)
    A = P.Stencil5.from_problem(p)
    G = P.ainv_setup(A, 0.05)
    for w in (-1, 65):
        with pytest.raises(P.PcgaError):
            G.layout_info(w)
    assert G.layout_info(0) == G.layout_info(32)
