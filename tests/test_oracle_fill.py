"""Pins of the oracle's fixed-fill AINV (CPU): the second Bridson class of
Sec. 5, where the number of nonzeros in each row of the lower factor Z^T
(each column of Z) is set in advance.  Reading: a finished column keeps its
`fill` off-diagonal entries of largest magnitude (equal magnitudes: the row
nearer the diagonal first), and its pivot is formed from the capped column.

Checked against facts that do not come from the oracle: the closed form of
the 1-D Laplacian's inverse factor restricted to a band, Jacobi at fill 0,
the uncapped threshold factor when the cap never binds, the A-orthogonality
that defines each pivot, and a dense brute-force statement of the method on
tiny grids."""
import numpy as np
import pytest

from gen import orca
from tests._cases import const_periodic, laplace1d, mixed_sign_dominant

EPS = np.finfo(float).eps


def _dense_a(p):
    """Dense A from its five-point storage (symmetric by construction)."""
    n, nx = p.n, p.nx
    A = np.zeros((n, n))
    for k in range(n):
        i, j = k % nx, k // nx
        A[k, k] = p.diag[k]
        if i < nx - 1 or p.periodic:
            e = k + 1 if i < nx - 1 else k - nx + 1
            A[k, e] += p.ae[k]
            A[e, k] += p.ae[k]
        if j < p.ny - 1:
            A[k, k + nx] += p.an[k]
            A[k + nx, k] += p.an[k]
    return A


@pytest.mark.parametrize("fill", [1, 2, 5])
def test_fill_laplace1d_is_band_of_exact_factor(ora, fill):
    """tridiag(-1,2,-1): column j is e_j + z_{j-1} / p_{j-1}, so a capped
    z_{j-1} yields the exact entries k/j (1-indexed) on its rows; the largest
    are the nearest to the diagonal, so the capped factor is the exact one
    restricted to the band j - fill <= k <= j, with the exact pivots
    (k+1)/k (the pivot reads only the subdiagonal entry)."""
    n = 40
    F = ora.ainv_setup(laplace1d(n), 0.0, fill=fill)
    Z = F.dense_z()
    k = np.arange(1, n + 1)
    ref = np.triu(k[:, None] / k[None, :])
    band = np.triu(np.ones((n, n), dtype=bool)) & ~np.triu(np.ones((n, n), dtype=bool), fill + 1)
    assert np.array_equal(Z != 0, band)
    assert np.allclose(Z[band], ref[band], rtol=4 * n * EPS, atol=0)
    assert np.allclose(F.D, (k + 1) / k, rtol=4 * EPS, atol=0)


@pytest.mark.parametrize("make", [lambda: orca.orca_problem(37, 23, 5),
                                  lambda: const_periodic(9, 7)])
def test_fill_zero_is_jacobi(ora, make):
    """No off-diagonal entry survives: Z = I and D = diag(A) exactly, the
    diagonal preconditioner of eq. (11)-(12)."""
    p = make()
    F = ora.ainv_setup(p, 0.0, fill=0)
    assert F.nnz_off == 0
    assert np.array_equal(F.D, p.diag)


@pytest.mark.parametrize("tau", [0.05, 0.1])
def test_fill_not_binding_is_threshold_factor(ora, tau):
    """A cap at or above the longest column changes nothing: the factor is
    bitwise the threshold one."""
    p = orca.orca_problem(37, 23, 5)
    T = ora.ainv_setup(p, tau)
    longest = int(np.diff(T.colptr).max())
    for fill in (longest, longest + 3):
        F = ora.ainv_setup(p, tau, fill=fill)
        assert np.array_equal(F.colptr, T.colptr)
        assert np.array_equal(F.rowidx, T.rowidx)
        assert np.array_equal(F.val, T.val) and np.array_equal(F.D, T.D)
    # one below the longest column binds somewhere
    F = ora.ainv_setup(p, tau, fill=longest - 1)
    assert F.nnz_off < T.nnz_off
    assert int(np.diff(F.colptr).max()) == longest - 1


@pytest.mark.parametrize("fill", [1, 3, 6])
def test_fill_counts_and_pivots(ora, fill):
    """Every column keeps at most `fill` entries, and each pivot is the
    A-inner product of row j of A with the final (capped) column:
    p_j = a_j^T z_j.  A pivot formed before the cap would differ where the
    cap removed a grid neighbour of j (fill 1 always removes one)."""
    p = orca.orca_problem(24, 17, 8)
    F = ora.ainv_setup(p, 0.0, fill=fill)
    assert int(np.diff(F.colptr).max()) <= fill
    A = _dense_a(p)
    Z = F.dense_z()
    piv = np.einsum("jk,kj->j", A, Z)
    assert np.allclose(F.D, piv, rtol=1e-13, atol=0)
    assert (F.D > 0).all()


def _brute_force(A, tau, fill):
    """The method on dense arrays, right-looking: when step i starts z_i is
    final; cap it, form p_i = a_i^T z_i, then for every later column j with
    c_j = a_i^T z_j != 0 subtract (c_j / p_i) z_i, dropping each touched
    off-diagonal entry that is zero or below tau.  Row sums run over A's
    nonzero columns in increasing order, as the method states them."""
    n = A.shape[0]
    Z = np.eye(n)
    D = np.zeros(n)
    nzc = [np.flatnonzero(A[i]) for i in range(n)]

    def adot(i, j):
        s = 0.0
        for c in nzc[i]:
            if Z[c, j] != 0.0:
                s = s + A[i, c] * Z[c, j]
        return s

    for i in range(n):
        off = [r for r in range(i) if Z[r, i] != 0.0]
        if len(off) > fill:
            ranked = sorted(off, key=lambda r: (-abs(Z[r, i]), -r))
            for r in ranked[fill:]:
                Z[r, i] = 0.0
        D[i] = adot(i, i)
        assert D[i] > 0
        rows = [r for r in range(i + 1) if Z[r, i] != 0.0]
        for j in range(i + 1, n):
            c = adot(i, j)
            if c == 0.0:
                continue
            m = c / D[i]
            for r in rows:
                nv = Z[r, j] - m * Z[r, i]
                Z[r, j] = 0.0 if (nv == 0.0 or (r != j and abs(nv) < tau)) else nv
    return Z, D


@pytest.mark.parametrize("tau,fill", [(0.0, 1), (0.0, 2), (0.0, 4), (0.02, 2), (0.02, 3)])
@pytest.mark.parametrize("make", [lambda: orca.orca_problem(7, 6, 3),
                                  lambda: const_periodic(6, 5),
                                  lambda: mixed_sign_dominant(7, 6, True, 3),
                                  lambda: mixed_sign_dominant(8, 5, False, 4)])
def test_fill_matches_dense_brute_force(ora, make, tau, fill):
    p = make()
    A = _dense_a(p)
    Zr, Dr = _brute_force(A, tau, fill)
    F = ora.ainv_setup(p, tau, fill=fill)
    Z = F.dense_z()
    assert np.array_equal(Z != 0, Zr != 0)
    assert np.allclose(Z, Zr, rtol=1e-12, atol=0)
    assert np.allclose(F.D, Dr, rtol=1e-12, atol=0)


def _drop_when_final(A, tau):
    """The other timing of the drop rule: updates kept in full, small
    entries of a column removed only once the column is final."""
    n = A.shape[0]
    Z = np.eye(n)
    for i in range(n):
        for r in range(i):
            if Z[r, i] != 0.0 and abs(Z[r, i]) < tau:
                Z[r, i] = 0.0
        p = A[i] @ Z[:, i]
        for j in range(i + 1, n):
            c = A[i] @ Z[:, j]
            if c != 0.0:
                Z[:, j] -= (c / p) * Z[:, i]
    return Z


@pytest.mark.parametrize("tau", [0.005, 0.02, 0.05, 0.1])
@pytest.mark.parametrize("make", [lambda: orca.orca_problem(7, 6, 3),
                                  lambda: orca.orca_problem(9, 8, 11),
                                  lambda: const_periodic(6, 5),
                                  lambda: mixed_sign_dominant(7, 6, True, 3),
                                  lambda: mixed_sign_dominant(8, 5, False, 4)])
def test_threshold_factor_matches_dense_brute_force(ora, make, tau):
    """The plain threshold factor (no count cap) on 2-D grids against the
    dense right-looking restatement with a cap that never binds: the drop
    test after every column update, not only at the end, decides which
    entries survive (with a binding tau the two timings give different
    patterns on these grids)."""
    p = make()
    A = _dense_a(p)
    Zr, Dr = _brute_force(A, tau, A.shape[0])
    F = ora.ainv_setup(p, tau)
    Z = F.dense_z()
    assert np.array_equal(Z != 0, Zr != 0)
    assert np.allclose(Z, Zr, rtol=1e-12, atol=0)
    assert np.allclose(F.D, Dr, rtol=1e-12, atol=0)
    if tau >= 0.02:
        # the test tells the two timings apart on these grids
        assert not np.array_equal(Z != 0, _drop_when_final(A, tau) != 0)


def test_fill_rejects_negative(ora):
    with pytest.raises(ValueError):
        ora.ainv_setup(laplace1d(5), 0.0, fill=-1)
