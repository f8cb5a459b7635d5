"""Host check of the Z-to-Z^T value map of the FP64 Z sweep (no device).

The Z sweep reads the values of Z's table steps from Z^T's value array,
which stays in the memory-side cache, through a per-step map built on the
host (sell_shared_values in csrc/layout.cpp).  A mapped step's lanes must
read exactly the values Z stores (bitwise, zeros included) and never leave
Z^T's values plus the 64-zero block after them: the device dereferences
these positions.  Checked by a small C++ program built from the library's
host sources on grids of the test and headline sizes.
"""
import os
import subprocess

import numpy as np
import pytest

from gen import orca

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1210_1878_amd", "csrc")


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("mapcheck") / "layout_map_check")
    r = subprocess.run(["g++", "-std=c++17", "-O2", "-I", CSRC, "-I", os.path.join(ROOT, "include"),
                        "-I", "/opt/rocm/include", os.path.join(ROOT, "tests", "layout_map_check.cpp"),
                        os.path.join(CSRC, "layout.cpp"), os.path.join(CSRC, "ainv.cpp"), "-o", out],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    return out


@pytest.mark.parametrize("nx,ny,seed,tau,min_frac", [
    (64, 48, 3, 0.05, 0.9),
    (182, 149, orca.CONFIG_SEED_BASE + 1, 0.1, 0.99),
    (362, 292, 5, 0.01, 0.0),      # fill-heavy factor: few table slices
    (721, 510, 7, 0.05, 0.99),
    (1442, 1021, orca.CONFIG_SEED_BASE + 2, 0.05, 0.99),
])
def test_value_map_reads_z_values(checker, tmp_path, nx, ny, seed, tau, min_frac):
    p = orca.orca_problem(nx, ny, seed)
    f = tmp_path / "a5.bin"
    with open(f, "wb") as fh:
        for arr in (p.diag, p.ae, p.an):
            fh.write(np.ascontiguousarray(arr, dtype=np.float64).tobytes())
    r = subprocess.run([checker, str(nx), str(ny), str(int(p.periodic)), str(tau), str(f)],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr
    steps, mapped, mism, oob = map(int, r.stdout.split())
    assert mism == 0 and oob == 0
    assert steps == 0 or mapped >= min_frac * steps
