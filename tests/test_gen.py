"""Generator invariants: the operator is the SPD negation of eq. (10)."""
import math

import numpy as np
import pytest

from gen import orca
from tests._cases import stencil_reference


def _offdiag_ok(p):
    A = p.dense()
    assert np.array_equal(A, A.T)                      # symmetric, bitwise
    off = A - np.diag(np.diag(A))
    assert (off <= 0).all()                            # M-matrix sign pattern
    assert (A.sum(axis=1) >= -1e-12 * np.abs(A).max()).all()   # diagonally dominant rows
    return A


def test_box_small_structure():
    p = orca.box_problem(9, 7, seed=5)
    A = _offdiag_ok(p)
    # every face contributes to both diagonals: row sums are the boundary faces
    assert (np.diag(A) > 0).all()
    assert np.all(p.ae.reshape(7, 9)[:, -1] == 0)
    assert np.all(p.an.reshape(7, 9)[-1, :] == 0)


def test_box_constant_is_textbook_laplacian():
    p = orca.box_problem(8, 6, constant=True)
    x = np.random.default_rng(0).standard_normal(p.n)
    y = p.dense() @ x
    assert np.allclose(y, stencil_reference(8, 6, False, x), rtol=0, atol=1e-13)


def test_box_constant_eigenvalues_closed_form():
    # Dirichlet 5-point Laplacian: 4 sin^2(k pi / 2(nx+1)) + 4 sin^2(l pi / 2(ny+1))
    nx, ny = 8, 6
    p = orca.box_problem(nx, ny, constant=True)
    lam = np.sort(np.linalg.eigvalsh(p.dense()))
    k = np.arange(1, nx + 1)[:, None]
    l = np.arange(1, ny + 1)[None, :]
    ref = np.sort((4 * np.sin(k * np.pi / (2 * (nx + 1))) ** 2
                   + 4 * np.sin(l * np.pi / (2 * (ny + 1))) ** 2).ravel())
    assert np.allclose(lam, ref, rtol=0, atol=1e-12)


def test_manufactured_rhs_consistent():
    p = orca.box_problem()
    assert np.allclose(p.dense() @ p.u_star, p.b, rtol=0, atol=1e-12)


@pytest.mark.parametrize("nx,ny,seed", [(36, 30, 11), (182, 149, orca.CONFIG_SEED_BASE + 1)])
def test_orca_invariants(nx, ny, seed):
    p = orca.orca_problem(nx, ny, seed)
    n = p.n
    assert abs((~p.ocean).mean() - 0.35) <= 0.005
    # land rows are identity rows with zero rhs
    land = ~p.ocean
    assert np.all(p.diag[land] == 1.0) and np.all(p.b[land] == 0.0)
    assert np.all(p.ae[land] == 0.0) and np.all(p.an[land] == 0.0)
    # couplings only between two ocean cells, never across the north edge
    E = p.ae.reshape(ny, nx)
    oc = p.ocean.reshape(ny, nx)
    assert np.all(E[~(oc & np.roll(oc, -1, axis=1))] == 0.0)
    assert np.all(p.an.reshape(ny, nx)[-1] == 0.0)
    # periodic wrap entries exist where both ends are ocean
    wrap = oc[:, -1] & oc[:, 0]
    assert wrap.any() and np.all(E[wrap, -1] < 0)
    # off-diagonals <= 0 and diagonal dominance on ocean rows
    assert (p.ae <= 0).all() and (p.an <= 0).all()
    west = np.roll(E, 1, axis=1).ravel()
    south = np.zeros(n)
    south[nx:] = p.an[:-nx]
    rowsum = p.diag + p.ae + p.an + west + south
    assert (rowsum >= -1e-9 * p.diag).all()
    if n <= 2000:
        _offdiag_ok(p)


def test_orca_depth_and_anisotropy():
    """Depth is mapped to [500, 5500] m; E-W over N-S coupling grows like
    1/cos^2(phi) towards the pole (the alpha >> beta limit of Sec. 2)."""
    nx, ny = 182, 149
    rng = np.random.default_rng(3)
    lam = (np.arange(nx) + 0.5) * 2 * np.pi / nx
    phi = np.radians(-78.0 + (np.arange(ny) + 0.5) * 168.0 / ny)
    H = orca._bathymetry(nx, ny, lam, phi, rng)
    assert math.isclose(H.min(), 500.0) and math.isclose(H.max(), 5500.0)
    p = orca.orca_problem(nx, ny, orca.CONFIG_SEED_BASE + 1)
    E = -p.ae.reshape(ny, nx)
    N = -p.an.reshape(ny, nx)
    both = (E > 0) & (N > 0)
    ratio = np.where(both, E / np.where(N > 0, N, 1), np.nan)
    r_eq = np.nanmedian(ratio[ny // 2 - 5: ny // 2 + 5])
    r_pole = np.nanmedian(ratio[-6:-2])
    assert r_pole > 50 * r_eq


def test_generator_deterministic():
    a = orca.orca_problem(50, 40, 7)
    b = orca.orca_problem(50, 40, 7)
    for f in ("diag", "ae", "an", "b"):
        assert np.array_equal(getattr(a, f), getattr(b, f))


def test_ensemble_shapes():
    ens = orca.ensemble_problems(count=3)
    for p in ens:
        assert 182 <= p.nx <= 362 and 149 <= p.ny <= 292
        assert p.B.shape == (4, p.n)
