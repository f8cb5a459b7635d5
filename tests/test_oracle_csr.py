"""Pins of the oracle on general sparse SPD matrices in CSR (CPU only).

The comparison of Sec. 5 also uses a matrix that does not come from the
grid; the oracle's CSR entry points run the same A-orthogonalisation and
Algorithm 1 on such a matrix.  Pinned by: the five-point operator written as
CSR reproduces the grid path bit for bit (same operations in the same order);
dense algebra on seeded unstructured matrices (exact inverse factor at drop
tolerance 0, Jacobi at infinity, the Krylov minimiser, the dense solution
within the condition-number bound); input validation.
"""
import numpy as np
import pytest

from gen import orca
from gen.unstructured import csr_from_grid, unstructured_problem
from tests._cases import cholesky_ainv

EPS = np.finfo(np.float64).eps


@pytest.mark.parametrize("mk,tau", [
    (lambda: orca.orca_problem(37, 23, 5, land_frac=0.2), 0.05),
    (lambda: orca.box_problem(24, 18), 0.1),
    (lambda: orca.orca_problem(3, 7, 3, land_frac=0.2), 0.0),
])
def test_csr_path_equals_grid_path_bitwise(ora, mk, tau):
    p = mk()
    C = csr_from_grid(p)
    x = np.random.default_rng(3).standard_normal(p.n)
    assert np.array_equal(ora.spmv(p, x), ora.spmv(C, x))
    F1, F2 = ora.ainv_setup(p, tau), ora.ainv_setup(C, tau)
    for a, b in ((F1.colptr, F2.colptr), (F1.rowidx, F2.rowidx), (F1.val, F2.val), (F1.D, F2.D)):
        assert np.array_equal(a, b)
    G1, G2 = ora.ainv_setup(p, 0.01, fill=3), ora.ainv_setup(C, 0.01, fill=3)
    assert np.array_equal(G1.val, G2.val) and np.array_equal(G1.rowidx, G2.rowidx)
    r1, r2 = ora.pcg(p, F1, tol=1e-10), ora.pcg(C, F2, tol=1e-10)
    assert r1.iters == r2.iters and np.array_equal(r1.x, r2.x) and np.array_equal(r1.hist, r2.hist)


@pytest.mark.parametrize("kind", ["laplacian", "mixed"])
def test_generator_invariants(kind):
    P = unstructured_problem(1500, 21, kind=kind)
    M = P.dense()
    assert np.array_equal(M, M.T)
    assert np.linalg.eigvalsh(M).min() > 0.0
    deg = np.diff(P.rowptr)
    assert deg.max() >= deg.min() + 4          # irregular: not a grid stencil
    for k in range(P.n):
        c = P.col[P.rowptr[k]:P.rowptr[k + 1]]
        assert np.all(np.diff(c) > 0) and k in c
    off = M - np.diag(np.diag(M))
    if kind == "laplacian":
        assert off.max() <= 0.0 and np.all(M.sum(axis=1) >= -1e-12)
    else:
        assert off.max() > 0.0 and off.min() < 0.0
        dd, rs = np.diag(M), np.abs(off).sum(axis=1)
        # irreducibly diagonally dominant (sums compared up to their rounding)
        assert np.all(dd >= rs * (1 - 1e-12)) and np.any(dd > rs + 0.5)
    assert np.array_equal(unstructured_problem(1500, 21, kind=kind).val, P.val)


def test_csr_spmv_against_dense(ora):
    P = unstructured_problem(900, 5, kind="mixed")
    M = P.dense()
    x = np.random.default_rng(2).standard_normal(P.n)
    y = ora.spmv(P, x)
    bound = 8 * EPS * (np.abs(M) @ np.abs(x))
    assert np.all(np.abs(y - M @ x) <= bound)


@pytest.mark.parametrize("kind", ["laplacian", "mixed"])
def test_csr_ainv_tau0_is_exact_inverse_factor(ora, kind):
    P = unstructured_problem(300, 8, kind=kind)
    M = P.dense()
    F = ora.ainv_setup(P, 0.0)
    Z = F.dense_z()
    assert np.allclose(np.tril(Z, -1), 0.0) and np.allclose(np.diag(Z), 1.0)
    ZtAZ = Z.T @ M @ Z
    assert np.linalg.norm(ZtAZ - np.diag(F.D)) <= 1e-12 * np.linalg.norm(ZtAZ)
    Zc, Dc = cholesky_ainv(M)
    assert np.allclose(Z, Zc, rtol=1e-9, atol=1e-12) and np.allclose(F.D, Dc, rtol=1e-10)
    Minv = Z @ np.diag(1.0 / F.D) @ Z.T
    assert np.linalg.norm(Minv @ M - np.eye(P.n)) <= 1e-9
    r = ora.pcg(P, F, tol=1e-10)
    assert r.iters == 1 and r.hist[1] <= 1e-12


def test_csr_ainv_inf_is_jacobi(ora):
    P = unstructured_problem(500, 9)
    F = ora.ainv_setup(P, np.inf)
    assert F.nnz_off == 0 and np.array_equal(F.D, P.diag())


@pytest.mark.parametrize("kind", ["laplacian", "mixed"])
def test_csr_pcg_dense_solution_and_krylov(ora, kind):
    P = unstructured_problem(1200, 17, kind=kind)
    M = P.dense()
    xs = np.linalg.solve(M, P.b)
    ev = np.linalg.eigvalsh(M)
    kappa = ev.max() / ev.min()
    F = ora.ainv_setup(P, 0.05)
    r = ora.pcg(P, F, tol=1e-10)
    assert r.status == 0 and r.hist[-1] <= 1e-10
    assert np.linalg.norm(r.x - xs) <= kappa * 1e-10 * np.linalg.norm(xs)
    # x_m minimises the A-norm error over the preconditioned Krylov space
    Pm = F.dense_z() @ np.diag(1.0 / F.D) @ F.dense_z().T
    K = [Pm @ P.b]
    for m in range(1, 5):
        V = np.array(K).T
        c = np.linalg.solve(V.T @ M @ V, V.T @ P.b)
        xm = ora.pcg(P, F, tol=0.0, maxit=m).x
        assert np.linalg.norm(xm - V @ c) <= 1e-9 * np.linalg.norm(xs)
        K.append(Pm @ (M @ K[-1]))
    # AINV needs fewer iterations than the diagonal preconditioner
    assert r.iters < ora.pcg(P, ora.ainv_setup(P, np.inf), tol=1e-10).iters


def test_csr_validation(ora):
    P = unstructured_problem(200, 4)
    bad = [
        ("asymmetric value", lambda Q: Q.val.__setitem__(1, Q.val[1] * 1.5)),
        ("unsorted row", lambda Q: Q.col.__setitem__(slice(0, 2), Q.col[0:2][::-1])),
        ("non-positive diagonal", lambda Q: Q.val.__setitem__(
            int(np.nonzero(Q.col[:Q.rowptr[1]] == 0)[0][0]), -1.0)),
    ]
    for what, spoil in bad:
        Q = unstructured_problem(200, 4)
        spoil(Q)
        with pytest.raises(ora.OracleError) as e:
            ora.ainv_setup(Q, 0.1)
        assert e.value.status == ora.EINVAL, what
    F = ora.ainv_setup(P, 0.1)
    assert F.n == P.n
