"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Each test names the passage or the closed form it relies on.  None of them
re-types the oracle's own loops: they use closed forms (Propositions 1 and 3,
the 5-point Laplacian spectrum, the CG bound eq. (9)), dense factorizations
and Krylov-subspace optimality computed independently with numpy.
"""
import math

import numpy as np
import pytest

from gen import orca
from tests._cases import (cholesky_ainv, const_periodic, laplace1d, stencil_reference,
                          tridiag_problem)


# --------------------------------------------------------------------------
# operator product
# --------------------------------------------------------------------------
@pytest.mark.parametrize("periodic", [False, True])
def test_spmv_textbook_stencil(ora, periodic):
    """Constant 5-point Laplacian (Sec. 3, eq. (10) with unit faces)."""
    nx, ny = 11, 7
    if periodic:
        p = const_periodic(nx, ny)
    else:
        p = orca.box_problem(nx, ny, constant=True)
    x = np.random.default_rng(1).standard_normal(p.n)
    y = ora.spmv(p, x)
    assert np.allclose(y, stencil_reference(nx, ny, periodic, x), rtol=0, atol=1e-13)


def test_spmv_matches_dense_orca(ora):
    p = orca.orca_problem(24, 18, 4)
    x = np.random.default_rng(2).standard_normal(p.n)
    A = p.dense()
    assert np.allclose(ora.spmv(p, x), A @ x, rtol=1e-14, atol=1e-10 * np.abs(A).max())


# --------------------------------------------------------------------------
# AINV
# --------------------------------------------------------------------------
def test_ainv_laplace1d_closed_form(ora):
    """tridiag(-1,2,-1): the exact inverse factor has Z[k,j] = k/j (1-indexed,
    k <= j) and pivots p_k = (k+1)/k (Cholesky of the 1-D Laplacian)."""
    n = 40
    p = laplace1d(n)
    F = ora.ainv_setup(p, 0.0)
    Z = F.dense_z()
    k = np.arange(1, n + 1)
    ref = np.triu(k[:, None] / k[None, :])
    eps = np.finfo(float).eps
    # each column inherits the rounding of the previous one: <= ~3 ulp/step
    assert np.allclose(Z, ref, rtol=4 * n * eps, atol=0)
    assert np.allclose(F.D, (k + 1) / k, rtol=4 * eps, atol=0)


@pytest.mark.parametrize("tau", [0.1000001, 0.3000001, 0.4500001])
def test_ainv_laplace1d_threshold_pattern(ora, tau):
    """With a drop tolerance tau < 1/2 the kept set is exactly
    {(k, j): k/j >= tau}: column j is updated once, from column j-1; the
    subdiagonal entry (j-1)/j >= 1/2 always survives, so every pivot stays
    exact, and the kept entries of z_{j-1} are the only ones that can stay
    above tau after scaling by (j-1)/j."""
    n = 30
    F = ora.ainv_setup(laplace1d(n), tau)
    Z = F.dense_z()
    k = np.arange(1, n + 1)
    ref = np.triu(k[:, None] / k[None, :])
    keep = (ref >= tau)
    assert np.array_equal(Z != 0, keep)
    assert np.allclose(Z[keep], ref[keep], rtol=4 * n * np.finfo(float).eps, atol=0)


def test_ainv_tie_is_kept(ora):
    """Entry Z[1,2] of the 1-D Laplacian is exactly 1/2 in floating point;
    an entry equal to the tolerance is kept (the drop test is |z| < tau)."""
    F = ora.ainv_setup(laplace1d(4), 0.5)
    Z = F.dense_z()
    assert Z[0, 1] == 0.5
    assert Z[0, 2] == 0.0  # 1/3 < 1/2


def _prop3_inverse_factor(t_diag, t_off):
    """Proposition 3: for the bidiagonal Cholesky factor U of a diagonally
    dominant tridiagonal T, column k of Z = U^-1 is
      z_{k-i,k} = (-1)^i / u_kk * prod_{r=1..i} u_{k-r,k-r+1} / u_{k-r,k-r}.
    U is obtained from the textbook tridiagonal Cholesky recurrence."""
    n = len(t_diag)
    u = np.zeros(n)        # u_kk
    v = np.zeros(n)        # u_{k,k+1}
    for k in range(n):
        prev = v[k - 1] ** 2 if k > 0 else 0.0
        u[k] = math.sqrt(t_diag[k] - prev)
        if k < n - 1:
            v[k] = t_off[k] / u[k]
    Zp = np.zeros((n, n))
    for k in range(n):
        Zp[k, k] = 1.0 / u[k]
        prod = 1.0
        for i in range(1, k + 1):
            prod *= v[k - i] / u[k - i]
            Zp[k - i, k] = (-1) ** i / u[k] * prod
    return Zp, u


def test_ainv_matches_prop3_closed_form(ora):
    """AINV of a diagonally dominant tridiagonal matrix = Prop. 3's U^-1,
    rescaled to a unit diagonal; D = diag(U)^2."""
    rng = np.random.default_rng(7)
    n = 25
    off = -rng.uniform(0.5, 1.5, n)
    off[-1] = 0.0
    diag = np.abs(off) + np.abs(np.concatenate([[0.0], off[:-1]])) + rng.uniform(0.05, 0.5, n)
    p = tridiag_problem(diag, off)
    Zp, u = _prop3_inverse_factor(diag, off)
    F = ora.ainv_setup(p, 0.0)
    assert np.allclose(F.dense_z(), Zp * u[None, :], rtol=1e-13, atol=1e-300)
    assert np.allclose(F.D, u ** 2, rtol=1e-14)
    # magnitudes strictly decrease away from the diagonal (Prop. 3)
    Z = F.dense_z()
    for k in range(1, n):
        col = np.abs(Z[: k + 1, k])[::-1]
        assert np.all(np.diff(col) < 0)


def test_fsai_band_is_truncated_exact_factor(ora):
    """Sec. 3 scheme: the band-q factor of T equals the exact inverse factor of
    T with entries j > i+q removed, and D is exact (Prop. 2-3 make the
    dropped set the smallest entries)."""
    rng = np.random.default_rng(8)
    n = 30
    off = -rng.uniform(0.5, 1.5, n)
    off[-1] = 0.0
    diag = np.abs(off) + np.abs(np.concatenate([[0.0], off[:-1]])) + rng.uniform(0.05, 0.5, n)
    p = tridiag_problem(diag, off)
    Zp, u = _prop3_inverse_factor(diag, off)
    exact = Zp * u[None, :]
    for q in (1, 2, 4):
        F, _ = ora.fsai_band(p, q)
        Zb = F.dense_z()
        i, j = np.indices((n, n))
        trunc = np.where((j - i <= q), exact, 0.0)
        assert np.allclose(Zb, trunc, rtol=1e-13, atol=1e-300)
        assert np.allclose(F.D, u ** 2, rtol=1e-14)


def test_fsai_band_uses_only_ew_tridiagonal_part(ora):
    """T keeps |col-row| <= 1 of A: for a 2-D grid the factor only sees the
    east-west couplings inside each row of the grid (no wrap, no N-S)."""
    p = orca.orca_problem(20, 12, 9)
    F, _ = ora.fsai_band(p, 3)
    A = p.dense()
    n = p.n
    T = np.zeros_like(A)
    for k in range(n):
        for c in (k - 1, k, k + 1):
            if 0 <= c < n:
                T[k, c] = A[k, c]
    Zc, Dc = cholesky_ainv(T)
    i, j = np.indices((n, n))
    trunc = np.where((j - i <= 3), Zc, 0.0)
    assert np.allclose(F.dense_z(), trunc, rtol=1e-12, atol=1e-14)
    assert np.allclose(F.D, Dc, rtol=1e-12)


@pytest.mark.parametrize("which", ["box", "orca", "periodic"])
def test_ainv_tau0_is_exact_inverse_factor(ora, which):
    """tau = 0 keeps every nonzero: Z D^-1 Z^T = A^-1 and Z^T A Z = D, and Z
    is the unit-diagonal rescaling of L^-T from a dense Cholesky A = L L^T."""
    if which == "box":
        p = orca.box_problem(7, 5, seed=3)
    elif which == "orca":
        p = orca.orca_problem(12, 9, 21)
    else:
        p = const_periodic(6, 4)
    A = p.dense()
    F = ora.ainv_setup(p, 0.0)
    Z = F.dense_z()
    Zc, Dc = cholesky_ainv(A)
    assert np.allclose(Z, Zc, rtol=1e-11, atol=1e-12)
    assert np.allclose(F.D, Dc, rtol=1e-12)
    ZAZ = Z.T @ A @ Z
    scale = np.abs(ZAZ).max()
    assert np.abs(ZAZ - np.diag(F.D)).max() <= 1e-13 * scale
    assert np.allclose(Z @ np.diag(1 / F.D) @ Z.T, np.linalg.inv(A), rtol=1e-10,
                       atol=1e-12 * np.abs(np.linalg.inv(A)).max())
    assert (Z >= -1e-15).all()       # A is an M-matrix: its inverse factor is >= 0
    # exact preconditioner: PCG converges in one iteration
    r = ora.pcg(p, F, tol=1e-12, maxit=5)
    assert r.iters == 1


def test_ainv_tau_inf_is_jacobi(ora):
    """tau = inf drops every off-diagonal: Z = I, D = diag(A) exactly
    (NEMO's diagonal preconditioner M = diag(A), eq. (11)-(12))."""
    p = orca.orca_problem(30, 20, 5)
    F = ora.ainv_setup(p, np.inf)
    assert F.nnz_off == 0
    assert np.array_equal(F.D, p.diag)


def test_ainv_breakdown_on_indefinite(ora):
    """p_i <= 0 is reported (existence holds only for M/H-matrices)."""
    p = laplace1d(6)
    p.diag = p.diag.copy()
    p.diag[3] = 0.5           # row 3 no longer dominant: pivot turns negative
    with pytest.raises(ora.OracleError) as e:
        ora.ainv_setup(p, 0.0)
    assert e.value.status == ora.EBREAKDOWN


def test_ainv_threshold_properties(ora):
    """For any tau: unit upper Z, every stored entry >= tau in magnitude,
    pivots positive; ZtAZ has unit-scaled diagonal equal to D on columns
    that received no dropping."""
    p = orca.orca_problem(40, 30, 13)
    for tau in (0.02, 0.1, 0.3):
        F = ora.ainv_setup(p, tau)
        assert (np.abs(F.val) >= tau).all()
        assert (F.rowidx < np.repeat(np.arange(p.n), np.diff(F.colptr))).all()
        assert (F.D > 0).all()
    # pattern shrinks as tau grows
    nnz = [ora.ainv_setup(p, t).nnz_off for t in (0.0, 0.02, 0.1, 0.3)]
    assert nnz == sorted(nnz, reverse=True)


def test_prec_apply_dense(ora):
    p = orca.orca_problem(16, 12, 3)
    F = ora.ainv_setup(p, 0.1)
    Z = F.dense_z()
    r = np.random.default_rng(4).standard_normal(p.n)
    ref = Z @ ((Z.T @ r) / F.D)
    assert np.allclose(ora.prec_apply(F, r), ref, rtol=1e-13, atol=1e-13 * np.abs(ref).max())
    assert np.allclose(ora.zt_apply(F, r), (Z.T @ r) / F.D, rtol=1e-13, atol=1e-14)


# --------------------------------------------------------------------------
# PCG (Algorithm 1)
# --------------------------------------------------------------------------
def test_pcg_iterates_are_krylov_optimal(ora):
    """In exact arithmetic PCG's x_m minimises the A-norm error over
    x0 + span{P r0, (PA) P r0, ..., (PA)^(m-1) P r0}.  Checked against a dense
    Galerkin solve on that subspace; this fails if the direction update used
    r instead of the preconditioned s, or if P were applied wrongly."""
    p = orca.orca_problem(14, 10, 17)
    A = p.dense()
    F = ora.ainv_setup(p, 0.1)
    Z = F.dense_z()
    P = Z @ np.diag(1 / F.D) @ Z.T
    # on the ocean block the preconditioner is far from Jacobi
    oc = p.ocean
    Po = P[np.ix_(oc, oc)]
    assert np.abs(Po - np.diag(1 / p.diag[oc])).max() > 0.05 * np.abs(Po).max()
    b = p.b
    r0 = b.copy()
    for m in range(1, 7):
        V = [P @ r0]
        for _ in range(m - 1):
            V.append(P @ (A @ V[-1]))
        V = np.linalg.qr(np.array(V).T)[0]
        y = np.linalg.solve(V.T @ A @ V, V.T @ b)
        x_ref = V @ y
        res = ora.pcg(p, F, b=b, tol=0.0, maxit=m)
        assert res.iters == m
        assert np.linalg.norm(res.x - x_ref) <= 1e-9 * np.linalg.norm(x_ref)


def test_pcg_error_monotone_and_scalars_positive(ora):
    p = orca.orca_problem(18, 12, 23)
    A = p.dense()
    xs = np.linalg.solve(A, p.b)
    F = ora.ainv_setup(p, 0.1)
    errs = []
    for m in range(0, 25):
        x = ora.pcg(p, F, tol=0.0, maxit=m).x if m else np.zeros(p.n)
        e = x - xs
        errs.append(math.sqrt(e @ A @ e))
    assert all(b <= a * (1 + 1e-12) for a, b in zip(errs, errs[1:]))
    r = ora.pcg(p, F, tol=1e-10, scalars=True)
    assert r.status == ora.OK and (r.alphas > 0).all() and (r.betas > 0).all()


@pytest.mark.parametrize("tau", [0.1, np.inf])
def test_pcg_dense_solution(ora, tau):
    """||x - x*|| / ||x*|| <= kappa_2(A) * tol (x* from a dense Cholesky)."""
    import scipy.linalg as sla
    p = orca.orca_problem(20, 15, 31)
    A = p.dense()
    xs = sla.cho_solve(sla.cho_factor(A), p.b)
    kappa = np.linalg.cond(A)
    r = ora.pcg(p, ora.ainv_setup(p, tau), tol=1e-10)
    assert r.status == ora.OK
    assert r.hist[-1] <= 1e-10 and r.hist[-2] > 1e-10
    assert np.linalg.norm(r.x - xs) <= kappa * 1e-10 * np.linalg.norm(xs)
    true = np.linalg.norm(p.b - A @ r.x) / np.linalg.norm(p.b)
    assert true <= 2e-10


def test_pcg_manufactured_solution(ora):
    """64x48 box, tau=0.1, tol=1e-10: error against the smooth u* is within
    kappa_2 * tol."""
    p = orca.box_problem()
    lam = np.linalg.eigvalsh(p.dense())
    kappa = lam[-1] / lam[0]
    r = ora.pcg(p, ora.ainv_setup(p, 0.1), tol=1e-10)
    assert r.status == ora.OK
    err = np.linalg.norm(r.x - p.u_star) / np.linalg.norm(p.u_star)
    assert err <= kappa * 1e-10


def _lanczos_extremes(alphas, betas):
    """Lanczos tridiagonal from CG coefficients: T_kk = 1/a_k + b_{k-1}/a_{k-1},
    T_{k,k+1} = sqrt(b_k)/a_k."""
    m = len(alphas)
    T = np.zeros((m, m))
    for k in range(m):
        T[k, k] = 1.0 / alphas[k] + (betas[k - 1] / alphas[k - 1] if k > 0 else 0.0)
        if k < m - 1:
            T[k, k + 1] = T[k + 1, k] = math.sqrt(betas[k]) / alphas[k]
    ev = np.linalg.eigvalsh(T)
    return ev[0], ev[-1]


def test_cg_constant_laplacian_spectrum_and_bound(ora):
    """Constant 5-point Dirichlet Laplacian on 64x48: eigenvalues
    4 sin^2(k pi/(2(nx+1))) + 4 sin^2(l pi/(2(ny+1))) give lambda_min=6.4448e-3,
    lambda_max=7.99356, kappa=1240.32.  With a constant diagonal, Jacobi-PCG is
    plain CG; the Lanczos matrix built from its alpha/beta must reproduce the
    extreme eigenvalues (scaled by 1/4), and the iteration count must respect
    the CG bound eq. (9): ||r||/||b|| <= 2 sqrt(kappa) rho^m with
    rho = (sqrt(kappa)-1)/(sqrt(kappa)+1)."""
    nx, ny = 64, 48
    lmin = 4 * math.sin(math.pi / (2 * (nx + 1))) ** 2 + 4 * math.sin(math.pi / (2 * (ny + 1))) ** 2
    lmax = (4 * math.sin(nx * math.pi / (2 * (nx + 1))) ** 2
            + 4 * math.sin(ny * math.pi / (2 * (ny + 1))) ** 2)
    kappa = lmax / lmin
    assert abs(lmin - 6.4448e-3) < 1e-7 and abs(lmax - 7.99356) < 1e-5
    assert abs(kappa - 1240.32) < 0.01
    p = orca.box_problem(nx, ny, constant=True)
    p.b = np.random.default_rng(5).standard_normal(p.n)
    F = ora.ainv_setup(p, np.inf)
    r = ora.pcg(p, F, tol=1e-10, scalars=True)
    assert r.status == ora.OK
    sk = math.sqrt(kappa)
    rho = (sk - 1) / (sk + 1)
    bound = math.ceil(math.log(1e-10 / (2 * sk)) / math.log(rho))
    assert bound == 481
    assert r.iters <= bound
    lo, hi = _lanczos_extremes(r.alphas, r.betas)
    assert abs(lo - lmin / 4) <= 1e-8 * lmin and abs(hi - lmax / 4) <= 1e-8 * lmax


def test_prop1_limit_matrix(ora):
    """Proposition 1: the pole limit of M^-1 A is tridiag(-1/2, 1, -1/2) with
    eigenvalues 1 + cos(k pi/(n+1)).  The exact condition number is
    cot^2(pi/(2(n+1))) (about 4(n+1)^2/pi^2; the paper's n^2/2 is the
    leading-order estimate).  Lanczos from the oracle's CG reproduces both
    extreme eigenvalues."""
    n = 60
    p = tridiag_problem(np.ones(n), np.full(n, -0.5), b=np.random.default_rng(6).standard_normal(n))
    lam = np.sort(np.linalg.eigvalsh(p.dense()))
    k = np.arange(1, n + 1)
    assert np.allclose(lam, np.sort(1 + np.cos(k * np.pi / (n + 1))), atol=1e-13)
    kappa = lam[-1] / lam[0]
    assert math.isclose(kappa, 1 / math.tan(math.pi / (2 * (n + 1))) ** 2, rel_tol=1e-9)
    r = ora.pcg(p, ora.ainv_setup(p, np.inf), tol=1e-12, scalars=True)
    lo, hi = _lanczos_extremes(r.alphas, r.betas)
    assert abs(lo - lam[0]) < 1e-9 and abs(hi - lam[-1]) < 1e-9


def test_pcg_zero_rhs_and_warm_start(ora):
    p = orca.orca_problem(20, 14, 2)
    F = ora.ainv_setup(p, 0.1)
    r0 = ora.pcg(p, F, b=np.zeros(p.n), x0=np.ones(p.n))
    assert r0.iters == 0 and np.all(r0.x == 0) and r0.hist[0] == 0.0
    full = ora.pcg(p, F, tol=1e-10)
    warm = ora.pcg(p, F, x0=full.x, tol=1e-10)
    assert warm.iters == 0
    assert ora.pcg(p, F, tol=1e-10, maxit=3).status == ora.NOCONV


def test_ainv_beats_jacobi_towards_pole(ora):
    """Table 2's trend: the approximate inverse needs fewer iterations than
    the diagonal preconditioner on the polar-anisotropic operator."""
    p = orca.orca_problem(182, 149, orca.CONFIG_SEED_BASE + 1)
    ia = ora.pcg(p, ora.ainv_setup(p, 0.1), tol=1e-10).iters
    ij = ora.pcg(p, ora.ainv_setup(p, np.inf), tol=1e-10).iters
    assert ia < 0.7 * ij


# --------------------------------------------------------------------------
# mixed precision refinement
# --------------------------------------------------------------------------
def test_mixed_refinement_reaches_fp64_residual(ora):
    p = orca.orca_problem(60, 45, 41)
    F = ora.ainv_setup(p, 0.1)
    m = ora.pcg_mixed(p, F, tol=1e-10, inner_tol=1e-5)
    assert m.status == ora.OK and m.outer >= 2
    A = p.dense()
    true = np.linalg.norm(p.b - A @ m.x) / np.linalg.norm(p.b)
    assert true <= 1e-10
    # same quantity, different summation order: agree to rounding level
    assert abs(true - m.outer_hist[-1]) <= 1e-3 * true + 1e-13
    # each outer step gains roughly inner_tol (contraction)
    h = m.outer_hist
    assert all(h[i + 1] < 1e-3 * h[i] for i in range(len(h) - 1))
    xs = np.linalg.solve(A, p.b)
    assert np.linalg.norm(m.x - xs) <= np.linalg.cond(A) * 1e-10 * np.linalg.norm(xs)


@pytest.mark.parametrize("nx,ny,seed,tau", [(60, 45, 41, 0.1), (182, 149, orca.CONFIG_SEED_BASE + 1, 0.1),
                                          (120, 90, 7, 0.05)])
def test_mixed_keep_direction_follows_one_pcg_run(ora, nx, ny, seed, tau):
    """Refinement with the direction kept across corrections (reliable
    updates, Sleijpen and van der Vorst 1996): in exact arithmetic the inner
    iterates are those of one PCG run of Algorithm 1 whose residual is
    replaced by b - A x at each correction, so the inner FP32 iterations add
    up to the FP64 PCG's count, whatever the segment length; the restarted
    form, which throws the Krylov space away at every correction, needs
    about 30-60% more.  A dropped or wrong beta at a correction turns the
    first into the second.  Each correction reduces the true residual by
    about the segment factor, and the solution solves the dense system."""
    p = orca.orca_problem(nx, ny, seed)
    F = ora.ainv_setup(p, tau)
    ref = ora.pcg(p, F, tol=1e-10)
    for delta in (0.3, 0.1, 0.01):
        k = ora.pcg_mixed(p, F, tol=1e-10, inner_tol=delta, keep=True, max_outer=200)
        r = ora.pcg_mixed(p, F, tol=1e-10, inner_tol=delta, keep=False, max_outer=200)
        assert k.status == ora.OK and k.outer_hist[-1] <= 1e-10
        assert abs(k.inner_total - ref.iters) <= 2
        assert r.inner_total >= 1.25 * ref.iters
        h = k.outer_hist
        # a run stops at max(delta, tol / h[i]) of its start
        assert all(h[i + 1] <= 3.0 * max(delta, 1e-10 / h[i]) * h[i] for i in range(len(h) - 1))
        # about one correction per factor delta of the 1e-10 reduction
        assert k.outer <= int(np.ceil(10.0 / -np.log10(delta))) + 3
    if p.n <= 3000:
        A = p.dense()
        true = np.linalg.norm(p.b - A @ k.x) / np.linalg.norm(p.b)
        assert true <= 1e-10
        xs = np.linalg.solve(A, p.b)
        assert np.linalg.norm(k.x - xs) <= np.linalg.cond(A) * 1e-10 * np.linalg.norm(xs)


def test_mixed_keep_first_segment_is_the_restarted_inner_run(ora):
    """From x0 = 0 the first inner run of both forms starts from the same r0
    and direction s0; with a segment factor below what is left to reach the
    target, the keep form's first run stops at tol / rel_0 = tol, so a single
    restarted correction with inner_tol = tol gives the same solution."""
    p = orca.orca_problem(40, 30, 9)
    F = ora.ainv_setup(p, 0.1)
    k = ora.pcg_mixed(p, F, tol=1e-6, inner_tol=1e-9, keep=True, max_outer=1)
    r = ora.pcg_mixed(p, F, tol=1e-6, inner_tol=1e-6, keep=False, max_outer=1)
    assert k.outer == r.outer == 1 and k.inner_total == r.inner_total
    assert np.array_equal(k.x, r.x)


def test_evaluation_order_builds_compute_the_same_method(ora):
    """The oracle's evaluation-order builds (reversed or blocked inner-product
    sums, fused multiply-adds) differ from the default build by rounding only:
    on the 182x149 grid their iterates after 15 iterations agree with the
    default build's to 1e-12 (relative), all stop at the same 1e-10 target,
    and each iterate is still the A-norm minimiser over the Krylov space on
    the 64x48 box (the default build's pin, repeated per build)."""
    p = orca.orca_problem(182, 149, orca.CONFIG_SEED_BASE + 1)
    F = ora.ainv_setup(p, 0.1)
    ref = ora.pcg(p, F, tol=0.0, maxit=15).x
    window = ora.stop_window(p, F, tol=1e-10)
    assert set(window) == {None} | set(ora.VARIANTS)
    for v in ora.VARIANTS:
        x = ora.pcg(p, F, tol=0.0, maxit=15, variant=v).x
        assert np.linalg.norm(x - ref) <= 1e-12 * np.linalg.norm(ref)
        r = ora.pcg(p, F, tol=1e-10, variant=v)
        assert r.status == 0 and r.hist[-1] <= 1e-10
        assert abs(r.iters - window[None]) <= 5
    pb = orca.box_problem()
    Fb = ora.ainv_setup(pb, 0.1)
    M = pb.dense()
    xs = np.linalg.solve(M, pb.b)
    for v in [None] + list(ora.VARIANTS):
        # x_3 minimises the A-norm error over x0 + K_3(P A, P r0), x0 = 0
        Pm = Fb.dense_z() @ np.diag(1.0 / Fb.D) @ Fb.dense_z().T
        K = [Pm @ pb.b]
        for _ in range(2):
            K.append(Pm @ (M @ K[-1]))
        V = np.array(K).T
        c = np.linalg.solve(V.T @ M @ V, V.T @ pb.b)
        x3 = ora.pcg(pb, Fb, tol=0.0, maxit=3, variant=v).x
        assert np.linalg.norm(x3 - V @ c) <= 1e-10 * np.linalg.norm(xs)


def test_mixed_inner_operator_forms(ora):
    """The mixed form's inner product q = A d on FP32 vectors: with FP64
    coefficients it is the FP64 five-point product rounded to FP32 once; with
    the operator in FP32 it is the same sum done in FP32 arithmetic on rounded
    coefficients (checked against numpy float32 operations in the same
    order).  Both mixed forms reach the FP64 target."""
    p = orca.orca_problem(37, 23, 5)
    d = np.random.default_rng(4).standard_normal(p.n).astype(np.float32)
    q64 = ora.spmv32(p, d, a32=False)
    assert np.array_equal(q64, ora.spmv(p, d.astype(np.float64)).astype(np.float32))
    q32 = ora.spmv32(p, d, a32=True)
    M = p.dense()
    for k in range(p.n):
        acc = np.float32(0.0)
        for c in np.nonzero(M[k])[0]:       # row k in increasing column order
            acc = np.float32(acc + np.float32(np.float32(M[k, c]) * d[c]))
        assert q32[k] == acc
    F = ora.ainv_setup(p, 0.05)
    for a32 in (False, True):
        m = ora.pcg_mixed(p, F, tol=1e-10, a32=a32)
        x = m.x
        assert np.linalg.norm(p.b - ora.spmv(p, x)) / np.linalg.norm(p.b) <= 1e-10
