"""Host side of the general sparse (CSR) operator path (no device needed).

The library's setup on a CSR matrix is the same A-orthogonalisation as the
oracle's, so the Z pattern, its values and D must be bit-for-bit equal
(the setup parity bar of the method); invalid CSR input is rejected.
"""
import ctypes

import numpy as np
import pytest

from gen import orca
from gen.unstructured import csr_from_grid, unstructured_problem


@pytest.fixture(scope="module")
def pkg():
    import paper_1210_1878_amd as P
    from paper_1210_1878_amd import _lib
    _lib.load()
    return P


def _csr(pkg, p):
    return pkg.CsrMatrix.from_problem(p)


@pytest.mark.parametrize("mk,tau,fill", [
    (lambda: unstructured_problem(3000, 31), 0.05, None),
    (lambda: unstructured_problem(3000, 32, kind="mixed"), 0.02, None),
    (lambda: unstructured_problem(2000, 33), 0.01, 4),
    (lambda: unstructured_problem(700, 34), 0.0, None),
    (lambda: csr_from_grid(orca.orca_problem(37, 23, 5)), 0.05, None),
])
def test_setup_bitwise_equal_to_oracle(pkg, ora, mk, tau, fill):
    p = mk()
    G = pkg.ainv_setup(_csr(pkg, p), tau, fill=fill)
    F = ora.ainv_setup(p, tau, fill=fill)
    colptr, rowidx, val, D = G.export()
    assert G.nnz_off == F.nnz_off
    assert np.array_equal(colptr, F.colptr)
    assert np.array_equal(rowidx.astype(np.int64), F.rowidx)
    assert np.array_equal(val.view(np.uint64), F.val.view(np.uint64))
    assert np.array_equal(D.view(np.uint64), F.D.view(np.uint64))


def test_grid_as_csr_setup_equals_grid_setup(pkg):
    p = orca.orca_problem(61, 40, 9)
    A5 = pkg.Stencil5.from_problem(p)
    Ga = pkg.ainv_setup(A5, 0.05).export()
    Gc = pkg.ainv_setup(_csr(pkg, csr_from_grid(p)), 0.05).export()
    for a, b in zip(Ga, Gc):
        assert np.array_equal(a, b)


def test_invalid_csr_rejected(pkg):
    from paper_1210_1878_amd import _lib
    base = unstructured_problem(300, 3)
    cases = []
    q = unstructured_problem(300, 3)
    q.val[1] *= 1.25                                  # not symmetric
    cases.append(q)
    q = unstructured_problem(300, 3)
    q.col[0], q.col[1] = q.col[1], q.col[0]           # columns not ascending
    cases.append(q)
    q = unstructured_problem(300, 3)
    d = int(np.nonzero(q.col[:q.rowptr[1]] == 0)[0][0])
    q.val[d] = 0.0                                    # zero diagonal
    cases.append(q)
    q = unstructured_problem(300, 3)
    q.rowptr = q.rowptr.copy()
    q.rowptr[5] = q.rowptr[6] + 1                     # rowptr not monotone
    cases.append(q)
    for q in cases:
        with pytest.raises(_lib.PcgaError) as e:
            pkg.ainv_setup(_csr(pkg, q), 0.1)
        assert e.value.status == _lib.EINVAL
    # the solver-side checks reject a mixed-precision CSR solver and a
    # factor of another size, before any device work
    A = _csr(pkg, base)
    G = pkg.ainv_setup(A, 0.1)
    L = _lib.load()
    nb = ctypes.c_size_t()
    cs = A.c_struct()
    assert L.pcga_workspace_bytes_csr(ctypes.byref(cs), G.handle, _lib.MIXED, 0,
                                      ctypes.byref(nb)) == _lib.EINVAL
    assert L.pcga_workspace_bytes_csr(ctypes.byref(cs), G.handle, _lib.FP64, 0,
                                      ctypes.byref(nb)) == _lib.OK and nb.value > 0
    other = pkg.ainv_setup(_csr(pkg, unstructured_problem(301, 3)), 0.1)
    assert L.pcga_workspace_bytes_csr(ctypes.byref(cs), other.handle, _lib.FP64, 0,
                                      ctypes.byref(nb)) == _lib.EINVAL
