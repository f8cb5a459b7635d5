"""The allocation-free FP64 solve (pcga_pcg_solve_noalloc) against pcga_pcg_solve.

Both run the same kernels on the same operator and factor; the allocation-free
call keeps its vectors, partial sums and control block in the library's static
device array instead of the solver's workspace and launches without graphs.
Checked through the C ABI on two calls in a row, the second on a smaller grid
(so the array still holds the first call's contents): iteration counts, the
residual history and the solution against pcga_pcg_solve (bit for bit, and at
the parity bar of the method: relative 1e-9, iterations within 2), true
residual at the 1e-10 target, and the FP64 oracle's natural stop.  A grid
larger than the array is rejected with ENOMEM before any device work.
"""
import ctypes
import sys

import numpy as np
import pytest

from gen import orca

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def say(*a):
    print("[no-alloc]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def pkg():
    if not torch.cuda.is_available():
        pytest.skip("no ROCm device")
    import paper_1210_1878_amd as P
    return P


def _solve_both(pkg, ora, p, tau):
    from paper_1210_1878_amd import _lib
    L = _lib.load()
    A = pkg.Stencil5.from_problem(p)
    S = pkg.Solver(A, pkg.ainv_setup(A, tau), "fp64", device="cuda:0")
    b = torch.from_numpy(p.b).cuda()
    x0 = torch.from_numpy(np.random.default_rng(5).standard_normal(p.n) * p.ocean).cuda()
    ref = S.solve(b, x0=x0, tol=1e-10)
    # the allocation-free call, straight through the C ABI on preallocated buffers
    x = x0.clone()
    cap = p.n + 1
    hist = np.zeros(cap)
    iters, hl, tr = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double()
    torch.cuda.synchronize()
    st = L.pcga_pcg_solve_noalloc(S.handle, ctypes.c_void_p(b.data_ptr()),
                                  ctypes.c_void_p(x.data_ptr()), 1e-10, -1, ctypes.byref(iters),
                                  hist.ctypes.data, cap, ctypes.byref(hl), ctypes.byref(tr))
    assert st == _lib.OK, L.pcga_last_error()
    return S, ref, x.cpu().numpy(), iters.value, hist[: hl.value], tr.value


@pytest.mark.parametrize("first,second", [
    (("orca182x149", lambda: orca.orca_problem(182, 149, orca.CONFIG_SEED_BASE + 1), 0.1),
     ("box64x48", lambda: orca.box_problem(), 0.1)),
])
def test_noalloc_matches_solve_twice(pkg, ora, first, second):
    for name, mk, tau in (first, second):
        p = mk()
        say(name, p.nx, p.ny, "tau", tau)
        S, ref, x, iters, hist, true = _solve_both(pkg, ora, p, tau)
        xr = ref.x.cpu().numpy()
        say(f"  iters solve={ref.iters} noalloc={iters} true relres={true:.3e}")
        assert iters == ref.iters
        assert np.array_equal(hist, ref.hist)
        assert np.array_equal(x, xr)   # same kernels, same reductions: bit for bit
        assert np.linalg.norm(x - xr) <= 1e-9 * np.linalg.norm(xr)
        assert true <= 1e-10 and abs(true - ref.true_relres) <= 1e-12
        F = ora.ainv_setup(p, tau)
        o = ora.pcg(p, F, b=p.b, x0=np.random.default_rng(5).standard_normal(p.n) * p.ocean,
                    tol=1e-10)
        assert abs(iters - o.iters) <= 2
        tr_ora = np.linalg.norm(p.b - ora.spmv(p, x)) / np.linalg.norm(p.b)
        assert tr_ora <= 1.05e-10


def test_noalloc_rejects_grid_beyond_limit(pkg):
    from paper_1210_1878_amd import _lib
    L = _lib.load()
    # diagonal preconditioner: a quick setup on a grid above the static limit
    nx, ny = 1200, 1100
    n = nx * ny
    assert 7 * 8 * n > _lib.NOALLOC_MAX_BYTES
    p = orca.Problem(nx, ny, False, np.full(n, 4.0), np.zeros(n), np.zeros(n),
                     np.ones(n, dtype=bool), np.ones(n))
    A = pkg.Stencil5.from_problem(p)
    S = pkg.Solver(A, pkg.ainv_setup(A, np.inf), "fp64", device="cuda:0")
    b = torch.ones(n, dtype=torch.float64, device="cuda:0")
    x = torch.full((n,), 7.0, dtype=torch.float64, device="cuda:0")
    torch.cuda.synchronize()
    iters = ctypes.c_int32(-5)
    st = L.pcga_pcg_solve_noalloc(S.handle, ctypes.c_void_p(b.data_ptr()),
                                  ctypes.c_void_p(x.data_ptr()), 1e-10, -1, ctypes.byref(iters),
                                  None, 0, None, None)
    say("beyond limit:", st, L.pcga_last_error())
    assert st == _lib.ENOMEM
    assert b"static scratch" in L.pcga_last_error()
    assert iters.value == -5
    assert bool(torch.all(x == 7.0))
