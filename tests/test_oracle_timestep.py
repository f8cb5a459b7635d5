"""Pins of the oracle's time-step functions (CPU): the right-hand side of
eq. (8) from face transports, the sea-surface update of eq. (1) and the first
guess of Algorithm 1.  Each is checked against facts that do not come from
the oracle itself: single-face impulses (the sign of each term of eq. (8) and
the closed and periodic faces), a face-by-face scatter formulation of the
same divergence, the telescoping of a closed basin's total, and closed forms."""
import numpy as np
import pytest

import oracle
from gen import orca


def _zeros(n):
    return [np.zeros(n) for _ in range(4)]


@pytest.mark.parametrize("periodic", [False, True])
def test_east_face_impulse(periodic):
    # b = -(delta_i(e2 Mu) - ...): a flux F out through the east face of k0
    # gives b[k0] = -F and b[east] = +F
    nx, ny = 5, 4
    e2u, mu, e1v, mv = _zeros(nx * ny)
    e2u[:] = 2.5
    k0 = 2 * nx + 1
    mu[k0] = 1.0
    b = oracle.ts_rhs(nx, ny, periodic, e2u, mu, e1v, mv)
    want = np.zeros(nx * ny)
    want[k0], want[k0 + 1] = -2.5, 2.5
    assert np.array_equal(b, want)


@pytest.mark.parametrize("periodic", [False, True])
def test_last_column_east_face(periodic):
    # the east face of i = nx-1 is the west face of i = 0 on a periodic grid,
    # closed otherwise
    nx, ny = 5, 4
    e2u, mu, e1v, mv = _zeros(nx * ny)
    e2u[:] = 1.0
    k0 = 1 * nx + nx - 1
    mu[k0] = 3.0
    b = oracle.ts_rhs(nx, ny, periodic, e2u, mu, e1v, mv)
    want = np.zeros(nx * ny)
    if periodic:
        want[k0], want[1 * nx] = -3.0, 3.0
    assert np.array_equal(b, want)


def test_north_face_impulse_and_closed_top():
    # the printed eq. (8) subtracts delta_j(e1 Mv): a flux through the north
    # face of k0 gives b[k0] = +F and b[north] = -F; the top row's north face
    # is closed
    nx, ny = 4, 3
    e2u, mu, e1v, mv = _zeros(nx * ny)
    e1v[:] = 3.0
    k0 = 0 * nx + 2
    mv[k0] = 1.0
    b = oracle.ts_rhs(nx, ny, True, e2u, mu, e1v, mv)
    want = np.zeros(nx * ny)
    want[k0], want[k0 + nx] = 3.0, -3.0
    assert np.array_equal(b, want)
    mv[:] = 0.0
    mv[(ny - 1) * nx + 1] = 5.0
    assert not np.any(oracle.ts_rhs(nx, ny, True, e2u, mu, e1v, mv))


def _scatter_rhs(nx, ny, periodic, e2u, mu, e1v, mv):
    """The same right-hand side assembled face by face: every open face adds
    its flux to one cell and subtracts it from the other."""
    bp = np.zeros(nx * ny)
    for j in range(ny):
        for i in range(nx):
            k = j * nx + i
            if i < nx - 1 or periodic:
                east = j * nx + (i + 1) % nx
                f = e2u[k] * mu[k]
                bp[k] += f          # outflow through the cell's east face
                bp[east] -= f       # inflow through the neighbour's west face
            if j < ny - 1:
                f = e1v[k] * mv[k]
                bp[k] -= f          # minus delta_j: outflow north counts negative
                bp[k + nx] += f
    return -bp


@pytest.mark.parametrize("nx,ny,periodic", [(9, 7, False), (9, 7, True), (24, 17, True)])
def test_matches_face_scatter(nx, ny, periodic):
    rng = np.random.default_rng(nx * 100 + ny + periodic)
    arrs = [rng.standard_normal(nx * ny) for _ in range(4)]
    b = oracle.ts_rhs(nx, ny, periodic, *arrs)
    ref = _scatter_rhs(nx, ny, periodic, *arrs)
    assert np.allclose(b, ref, rtol=0, atol=1e-14 * np.abs(ref).max())


def test_orca_transports_closed_basin():
    # land faces carry nothing, so land rows get b = 0, and the total over the
    # (periodic, closed north and south) basin telescopes to zero
    p = orca.orca_problem(182, 149, orca.CONFIG_SEED_BASE + 1)
    for t in (0, 7):
        e2u, mu, e1v, mv = orca.orca_transports(p, t, seed=11)
        b = oracle.ts_rhs(p.nx, p.ny, p.periodic, e2u, mu, e1v, mv)
        assert not np.any(b[~p.ocean])
        assert abs(b.sum()) <= 1e-13 * np.abs(b).sum()
        assert np.abs(b).max() > 0


def test_transports_vary_smoothly_in_time():
    p = orca.orca_problem(182, 149, orca.CONFIG_SEED_BASE + 1)
    m0 = orca.orca_transports(p, 10, seed=3)[1]
    m1 = orca.orca_transports(p, 11, seed=3)[1]
    m2 = orca.orca_transports(p, 12, seed=3)[1]
    step = np.linalg.norm(m1 - m0) / np.linalg.norm(m0)
    assert 0 < step < 0.1
    # second differences much smaller than first: linear extrapolation helps
    assert np.linalg.norm(m2 - 2 * m1 + m0) < 0.2 * np.linalg.norm(m1 - m0)


def test_eta_update_closed_form():
    eta_prev = np.array([1.0, 2.0, -0.5])
    D = np.array([0.5, -1.0, 0.0])
    assert np.array_equal(oracle.ts_eta(eta_prev, D, 0.25), np.array([0.75, 2.5, -0.5]))


def test_guess_closed_form():
    D1 = np.array([1.0, -2.0, 0.5])
    D2 = np.array([0.5, 1.0, 0.5])
    assert np.array_equal(oracle.ts_guess(D1, D2, 2.0, -1.0), np.array([1.5, -5.0, 0.5]))
    # c = 0 leaves D2 out entirely (a NaN there does not leak)
    assert np.array_equal(oracle.ts_guess(D1, np.full(3, np.nan), 2.0, 0.0), 2.0 * D1)
    assert np.array_equal(oracle.ts_guess(D1, None, 1.0, 0.0), D1)
