"""Device path vs the FP64 oracle, through the C ABI (needs an MI355X).

Bars (the method's problem statement): solutions iteration-matched to
relative 1e-9 in FP64, natural stopping iteration counts within +-2, true
residuals at the 1e-10 target; single kernels within a few ulp of the
oracle's operation, scaled by the magnitude of the terms they sum.
"""
import sys

import numpy as np
import pytest

from gen import orca
from tests._cases import const_periodic, laplace1d, tridiag_problem

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

EPS = np.finfo(np.float64).eps


def say(*a):
    print("[gpu-parity]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def pkg():
    if not torch.cuda.is_available():
        pytest.skip("no ROCm device")
    import paper_1210_1878_amd as P
    return P


CASES = {
    "box64x48": (lambda: orca.box_problem(), 0.1),
    "orca182x149": (lambda: orca.orca_problem(182, 149, orca.CONFIG_SEED_BASE + 1), 0.1),
    "orca182x149_jacobi": (lambda: orca.orca_problem(182, 149, orca.CONFIG_SEED_BASE + 1), np.inf),
    "orca37x23_ragged": (lambda: orca.orca_problem(37, 23, 5), 0.05),
    "periodic9x5_exact": (lambda: const_periodic(9, 5, b=np.random.default_rng(1).standard_normal(45)), 0.0),
    "line100": (lambda: laplace1d(100), 0.1),
    "orca3x7_min_periodic": (lambda: orca.orca_problem(3, 7, 3, land_frac=0.2), 0.1),
}

_cache = {}


def case(name):
    if name not in _cache:
        mk, tau = CASES[name]
        _cache[name] = (mk(), tau)
    return _cache[name]


def _abs_problem(p):
    q = orca.Problem(p.nx, p.ny, p.periodic, np.abs(p.diag), np.abs(p.ae), np.abs(p.an),
                     p.ocean, p.b)
    return q


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


@pytest.mark.parametrize("name", list(CASES))
def test_apply_a(pkg, ora, name):
    p, tau = case(name)
    say("apply_a", name, p.nx, p.ny)
    S = pkg.Solver(pkg.Stencil5.from_problem(p), pkg.ainv_setup(pkg.Stencil5.from_problem(p), tau))
    x = np.random.default_rng(11).standard_normal(p.n)
    y = S.apply_a(dev(x)).cpu().numpy()
    ref = ora.spmv(p, x)
    mag = ora.spmv(_abs_problem(p), np.abs(x))
    assert np.all(np.abs(y - ref) <= 8 * EPS * mag + 1e-300)


def check_stencil_step(pkg, ora, S, p, prec, seed, beta):
    """The fused first kernel of an iteration alone (pcga_step_stencil):
    d_new = s + beta d, q = A d_new and (d_new, q), element by element.
    d_new against the direction update of Algorithm 1 (one rounding of the
    fused form); q against the oracle's five-point product of the device's
    d_new (the FP64 coefficients; in the mixed form the product is rounded
    to FP32 once); (d_new, q) against the sum of the device's products within
    the bound of a recursive sum."""
    rng = np.random.default_rng(seed)
    s, d = rng.standard_normal(p.n), rng.standard_normal(p.n)
    if prec != "fp64":              # the FP32 kernel's inputs, exactly
        s = s.astype(np.float32).astype(np.float64)
        d = d.astype(np.float32).astype(np.float64)
        bt = float(np.float32(beta))
        u = float(np.finfo(np.float32).eps) / 2
    else:
        bt = beta
        u = EPS / 2
    dn, q, dq = S.step_stencil(dev(s), dev(d), beta)
    dn, q = dn.cpu().numpy(), q.cpu().numpy()
    d_ref = s + bt * d
    assert np.all(np.abs(dn - d_ref) <= 2 * u * (np.abs(s) + np.abs(bt * d)) + 1e-300)
    if prec != "fp64":
        assert np.array_equal(dn, dn.astype(np.float32).astype(np.float64))
    mag = ora.spmv(_abs_problem(p), np.abs(dn))
    if prec == "mixed_a32":
        # FP32 coefficients, FP32 sums: the oracle's FP32 product of the
        # device's d_new, within the bound of a 5-term FP32 sum
        q_ref = ora.spmv32(p, dn, a32=True).astype(np.float64)
        assert np.all(np.abs(q - q_ref) <= 12 * u * mag + 1e-300)
    else:
        q_ref = ora.spmv(p, dn)
        assert np.all(np.abs(q - q_ref) <= u * np.abs(q_ref) + 8 * EPS * mag + 1e-300)
    prods = dn * q
    gam = 1.01 * p.n * EPS
    assert abs(dq - np.sum(prods)) <= gam * np.sum(np.abs(prods)) + 1e-300
    return dn, q, dq


STENCIL_CASES = ["box64x48", "orca182x149", "orca37x23_ragged", "orca3x7_min_periodic",
                 "orca182x149_jacobi"]


@pytest.mark.parametrize("name", STENCIL_CASES)
@pytest.mark.parametrize("prec", ["fp64", "mixed", "mixed_a32"])
def test_fused_stencil_step(pkg, ora, name, prec):
    p, tau = case(name)
    say("fused stencil step", name, prec)
    A = pkg.Stencil5.from_problem(p)
    S = pkg.Solver(A, pkg.ainv_setup(A, tau), prec)
    for seed, beta in ((41, 0.37), (42, 0.0), (43, 1.93)):
        check_stencil_step(pkg, ora, S, p, prec, seed, beta)
    # the solver stays usable after the stand-alone launches
    if prec == "fp64":
        g = S.solve(dev(p.b), tol=1e-10)
        assert g.status == 0 and g.hist[-1] <= 1e-10
    with pytest.raises(Exception):
        S.step_stencil(dev(np.zeros(p.n)), dev(np.zeros(p.n)), -1.0)


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_apply_prec(pkg, ora, name, prec):
    p, tau = case(name)
    say("apply_prec", name, prec)
    A = pkg.Stencil5.from_problem(p)
    G = pkg.ainv_setup(A, tau)
    F = ora.ainv_setup(p, tau)
    S = pkg.Solver(A, G, prec)
    r = np.random.default_rng(12).standard_normal(p.n)
    t, s = S.apply_prec(dev(r))
    t, s = t.cpu().numpy(), s.cpu().numpy()
    t_ref = ora.zt_apply(F, r)
    s_ref = ora.z_apply(F, t_ref)
    Fa = ora.AInv(F.n, F.colptr, F.rowidx, np.abs(F.val), F.D)
    t_mag = ora.zt_apply(Fa, np.abs(r))
    s_mag = ora.z_apply(Fa, t_mag)
    u = 4 * EPS if prec == "fp64" else 4 * np.finfo(np.float32).eps
    width = max(8, int(np.diff(F.colptr).max()) + 2)
    assert np.all(np.abs(t - t_ref) <= width * u * t_mag + 1e-300)
    assert np.all(np.abs(s - s_ref) <= 2 * width * u * s_mag + 1e-300)


def test_wide_index_fallback(pkg, ora):
    """Grid rows longer than 65535 cells put Z entries beyond a 16-bit
    distance from their row: the solver keeps 32-bit columns there (and
    16-bit distances on ordinary grids); both formats match the oracle."""
    p = orca.box_problem(70000, 3, seed=5)
    q, tau = case("orca182x149")
    A = pkg.Stencil5.from_problem(p)
    G = pkg.ainv_setup(A, 0.1)
    F = ora.ainv_setup(p, 0.1)
    assert int(np.max(np.arange(p.n).repeat(np.diff(F.colptr)) - F.rowidx)) > 65535
    S = pkg.Solver(A, G, "fp64")
    say("wide index fallback: index bytes", S.index_bytes)
    assert S.index_bytes == 4
    Aq = pkg.Stencil5.from_problem(q)
    assert pkg.Solver(Aq, pkg.ainv_setup(Aq, tau), "fp64").index_bytes == 2
    assert pkg.Solver(Aq, pkg.ainv_setup(Aq, tau), "mixed").index_bytes == 2
    r = np.random.default_rng(13).standard_normal(p.n)
    t, s = S.apply_prec(dev(r))
    t_ref = ora.zt_apply(F, r)
    s_ref = ora.z_apply(F, t_ref)
    Fa = ora.AInv(F.n, F.colptr, F.rowidx, np.abs(F.val), F.D)
    t_mag = ora.zt_apply(Fa, np.abs(r))
    s_mag = ora.z_apply(Fa, t_mag)
    width = max(8, int(np.diff(F.colptr).max()) + 2)
    assert np.all(np.abs(t.cpu().numpy() - t_ref) <= width * 4 * EPS * t_mag + 1e-300)
    assert np.all(np.abs(s.cpu().numpy() - s_ref) <= 2 * width * 4 * EPS * s_mag + 1e-300)
    K = 30
    g = S.solve(dev(p.b), tol=0.0, maxit=K)
    o = ora.pcg(p, F, tol=0.0, maxit=K)
    assert g.iters == o.iters == K
    assert np.linalg.norm(g.x.cpu().numpy() - o.x) <= 1e-9 * np.linalg.norm(o.x)
    Sm = pkg.Solver(A, G, "mixed")
    assert Sm.index_bytes == 4
    tm, sm = Sm.apply_prec(dev(r))
    u32 = 4 * np.finfo(np.float32).eps
    assert np.all(np.abs(tm.cpu().numpy() - t_ref) <= width * u32 * t_mag + 1e-300)
    assert np.all(np.abs(sm.cpu().numpy() - s_ref) <= 2 * width * u32 * s_mag + 1e-300)


def _solve_pair(pkg, ora, p, tau, tol, maxit=None, x0=None, b=None):
    A = pkg.Stencil5.from_problem(p)
    G = pkg.ainv_setup(A, tau)
    F = ora.ainv_setup(p, tau)
    b = p.b if b is None else b
    S = pkg.Solver(A, G, "fp64")
    g = S.solve(dev(b), None if x0 is None else dev(x0), tol=tol, maxit=maxit)
    o = ora.pcg(p, F, b=b, x0=x0, tol=tol, maxit=maxit)
    return g, o, S


@pytest.mark.parametrize("name", list(CASES))
def test_pcg_iteration_matched(pkg, ora, name):
    p, tau = case(name)
    o0 = ora.pcg(p, ora.ainv_setup(p, tau), tol=1e-10)
    K = max(o0.iters, 1)
    say("pcg iteration-matched", name, "K =", K)
    g, o, _ = _solve_pair(pkg, ora, p, tau, tol=0.0, maxit=K)
    assert g.iters == o.iters == K
    xo = o.x
    assert np.linalg.norm(g.x.cpu().numpy() - xo) <= 1e-9 * np.linalg.norm(xo)
    # residual histories agree as well
    assert np.allclose(g.hist, o.hist, rtol=1e-6, atol=1e-14)


@pytest.mark.parametrize("width", [1, 8, 32, 64])
def test_pcg_other_slice_widths(pkg, ora, width):
    """Any sliced-ELL target width is the same method: iteration-matched
    solution and natural stop as with the default."""
    p, tau = case("orca182x149")
    say("pcg with slice width", width)
    A = pkg.Stencil5.from_problem(p)
    S = pkg.Solver(A, pkg.ainv_setup(A, tau), "fp64", slice_width=width)
    F = ora.ainv_setup(p, tau)
    K = ora.pcg(p, F, tol=1e-10).iters
    g = S.solve(torch.from_numpy(p.b).cuda(), tol=0.0, maxit=K)
    o = ora.pcg(p, F, tol=0.0, maxit=K)
    assert np.linalg.norm(g.x.cpu().numpy() - o.x) <= 1e-9 * np.linalg.norm(o.x)
    g = S.solve(torch.from_numpy(p.b).cuda(), tol=1e-10)
    assert g.status == 0 and abs(g.iters - K) <= 2


@pytest.mark.parametrize("width", [48, 64])
def test_wide_slices_tau001(pkg, ora, width):
    """Target widths up to 64 on the 182x149 factor at drop tolerance 0.01,
    whose one-lane-per-row slices have offset unions wider than one wavefront
    register: such slices must use per-lane indices.  The apply element by
    element and the iteration-matched solve against the oracle."""
    p = orca.orca_problem(182, 149, orca.CONFIG_SEED_BASE + 1)
    A = pkg.Stencil5.from_problem(p)
    G = pkg.ainv_setup(A, 0.01)
    F = ora.ainv_setup(p, 0.01)
    info = G.layout_info(width)
    say("wide slices, tau 0.01, width", width, info)
    assert info["zt"]["table_width_max"] <= 64 and info["z"]["table_width_max"] <= 64
    r = np.random.default_rng(15).standard_normal(p.n)
    Fa = ora.AInv(F.n, F.colptr, F.rowidx, np.abs(F.val), F.D)
    t_ref = ora.zt_apply(F, r)
    s_ref = ora.z_apply(F, t_ref)
    t_mag = ora.zt_apply(Fa, np.abs(r))
    s_mag = ora.z_apply(Fa, t_mag)
    wmax = int(np.diff(F.colptr).max()) + 2
    for prec in ("fp64", "mixed"):
        S = pkg.Solver(A, G, prec, slice_width=width)
        t, s = S.apply_prec(dev(r))
        u = 4 * EPS if prec == "fp64" else 4 * np.finfo(np.float32).eps
        assert np.all(np.abs(t.cpu().numpy() - t_ref) <= wmax * u * t_mag + 1e-300)
        assert np.all(np.abs(s.cpu().numpy() - s_ref) <= 2 * wmax * u * s_mag + 1e-300)
        if prec == "fp64":
            K = ora.pcg(p, F, tol=1e-10).iters
            g = S.solve(dev(p.b), tol=0.0, maxit=K)
            o = ora.pcg(p, F, tol=0.0, maxit=K)
            assert np.linalg.norm(g.x.cpu().numpy() - o.x) <= 1e-9 * np.linalg.norm(o.x)
            nat = S.solve(dev(p.b), tol=1e-10)
            assert nat.status == 0 and abs(nat.iters - K) <= 2
        S.close()


def test_autotuner_small(pkg):
    from paper_1210_1878_amd import autotune
    p, tau = case("orca182x149")
    A = pkg.Stencil5.from_problem(p)
    G = pkg.ainv_setup(A, tau)
    b = torch.from_numpy(p.b).cuda()
    r = autotune.tune_solver(A, G, b, "fp64", widths=(8, 16), blocks=(64, 256), chunks=(16, 32), reps=5)
    say("autotune", {k: r[k] for k in ("slice_width", "max_blocks", "chunk")})
    assert r["slice_width"] in (8, 16) and r["max_blocks"] in (64, 256) and r["chunk"] in (16, 32)
    assert len(r["table"]) == 4 and all(ms > 0 for _, _, ms in r["table"])
    S = pkg.Solver(A, G, "fp64", slice_width=r["slice_width"])
    S.tune(chunk=r["chunk"], max_blocks=r["max_blocks"])
    g = S.solve(b, tol=1e-10)
    assert g.status == 0 and g.hist[-1] <= 1e-10


@pytest.mark.parametrize("name", list(CASES))
def test_pcg_natural_stop(pkg, ora, name):
    p, tau = case(name)
    say("pcg natural stop", name)
    g, o, _ = _solve_pair(pkg, ora, p, tau, tol=1e-10)
    assert g.status == 0 and o.status == 0
    assert abs(g.iters - o.iters) <= 2
    assert g.hist[-1] <= 1e-10
    # FP64 true residual, recomputed independently with the oracle's product
    x = g.x.cpu().numpy()
    true = np.linalg.norm(p.b - ora.spmv(p, x)) / np.linalg.norm(p.b)
    assert true <= 1.05e-10
    assert abs(true - g.true_relres) <= 1e-3 * true + 1e-13


@pytest.mark.parametrize("name", ["box64x48", "orca182x149", "orca37x23_ragged"])
@pytest.mark.parametrize("form", ["mixed", "mixed_a32"])
def test_mixed_reaches_fp64_residual(pkg, ora, name, form):
    p, tau = case(name)
    say(form, name)
    A = pkg.Stencil5.from_problem(p)
    S = pkg.Solver(A, pkg.ainv_setup(A, tau), form)
    m = S.solve_mixed(dev(p.b), tol=1e-10, inner_tol=1e-5, max_outer=20)
    assert m.status == 0
    x = m.x.cpu().numpy()
    true = np.linalg.norm(p.b - ora.spmv(p, x)) / np.linalg.norm(p.b)
    assert true <= 1e-10
    # the same residual summed in two orders: equal to rounding level
    assert abs(true - m.true_relres) <= 1e-3 * true + 1e-13
    xo = ora.pcg(p, ora.ainv_setup(p, tau), tol=1e-12).x
    err = np.linalg.norm(x - xo) / np.linalg.norm(xo)
    say("  mixed outer", m.outer, "inner", m.inner_total, "rel err vs FP64 oracle", err)
    om = ora.pcg_mixed(p, ora.ainv_setup(p, tau), tol=1e-10, inner_tol=1e-5,
                       a32=(form == "mixed_a32"))
    assert abs(m.outer - om.outer) <= 1


@pytest.mark.parametrize("name", ["box64x48", "orca182x149", "orca37x23_ragged",
                                  "orca182x149_jacobi"])
@pytest.mark.parametrize("form", ["mixed", "mixed_a32"])
def test_mixed_keep_direction(pkg, ora, name, form):
    """Refinement with the direction kept across corrections: the FP64 true
    residual reaches the target, the corrections and the inner FP32
    iterations match the oracle's run of the same form, and the inner total
    stays near the FP64 PCG's count (the Krylov space survives corrections)."""
    p, tau = case(name)
    say(form, "keep", name)
    A = pkg.Stencil5.from_problem(p)
    S = pkg.Solver(A, pkg.ainv_setup(A, tau), form)
    m = S.solve_mixed(dev(p.b), tol=1e-10, refine="keep")
    assert m.status == 0
    x = m.x.cpu().numpy()
    true = np.linalg.norm(p.b - ora.spmv(p, x)) / np.linalg.norm(p.b)
    assert true <= 1e-10
    assert abs(true - m.true_relres) <= 1e-3 * true + 1e-13
    F = ora.ainv_setup(p, tau)
    om = ora.pcg_mixed(p, F, tol=1e-10, inner_tol=0.1, keep=True, max_outer=200,
                       a32=(form == "mixed_a32"))
    o64 = ora.pcg(p, F, tol=1e-10)
    say(f"  outer {m.outer} (oracle {om.outer}) inner {m.inner_total} (oracle {om.inner_total}, "
        f"FP64 PCG {o64.iters})")
    assert abs(m.outer - om.outer) <= 1
    assert abs(m.inner_total - om.inner_total) <= 3
    # FP32 rounding perturbs the run: within 15% of the FP64 count
    assert m.inner_total <= 1.15 * o64.iters + 3
    # restarted corrections of the same length lose the Krylov space
    r = S.solve_mixed(dev(p.b), tol=1e-10, inner_tol=0.1, max_outer=200)
    assert r.status == 0 and r.inner_total > m.inner_total


def test_mixed_keep_edges(pkg, ora):
    """Keep form: zero right-hand side, a converged first guess (nothing
    runs), a correction budget that ends early (NOCONV, x = x0 + the
    corrections made), and a second solve on the same solver."""
    p, tau = case("orca182x149")
    say("edge: keep form")
    A = pkg.Stencil5.from_problem(p)
    S = pkg.Solver(A, pkg.ainv_setup(A, tau), "mixed")
    z = S.solve_mixed(dev(np.zeros(p.n)), dev(np.ones(p.n)), refine="keep")
    assert z.status == 0 and z.outer == 0 and float(z.x.abs().max()) == 0.0
    full = S.solve_mixed(dev(p.b), tol=1e-10, refine="keep")
    assert full.status == 0
    warm = S.solve_mixed(dev(p.b), full.x, tol=1e-10, refine="keep")
    assert warm.status == 0 and warm.outer == 0 and warm.inner_total == 0
    assert torch.equal(warm.x, full.x)
    few = S.solve_mixed(dev(p.b), tol=1e-10, max_outer=2, refine="keep")
    assert few.status == 1 and few.outer == 2 and len(few.hist) == 3
    x = few.x.cpu().numpy()
    rel = np.linalg.norm(p.b - ora.spmv(p, x)) / np.linalg.norm(p.b)
    assert abs(rel - few.hist[-1]) <= 1e-3 * rel
    assert 1e-3 < rel < 0.05
    again = S.solve_mixed(dev(p.b), tol=1e-10, refine="keep")
    assert again.outer == full.outer and again.inner_total == full.inner_total
    assert torch.equal(again.x, full.x)


def test_edge_zero_rhs_and_warm_start(pkg, ora):
    p, tau = case("orca182x149")
    say("edge: zero rhs / warm start")
    A = pkg.Stencil5.from_problem(p)
    S = pkg.Solver(A, pkg.ainv_setup(A, tau))
    z = S.solve(dev(np.zeros(p.n)), dev(np.ones(p.n)))
    assert z.iters == 0 and z.status == 0 and float(z.x.abs().max()) == 0.0
    assert list(z.hist) == [0.0]
    full = S.solve(dev(p.b), tol=1e-10)
    warm = S.solve(dev(p.b), full.x, tol=1e-10)
    assert warm.iters == 0 and torch.equal(warm.x, full.x)
    few = S.solve(dev(p.b), tol=1e-10, maxit=3)
    assert few.status == 1 and few.iters == 3
    o3 = ora.pcg(p, ora.ainv_setup(p, tau), tol=1e-10, maxit=3)
    assert np.linalg.norm(few.x.cpu().numpy() - o3.x) <= 1e-12 * np.linalg.norm(o3.x)
    Sm = pkg.Solver(A, pkg.ainv_setup(A, tau), "mixed")
    zm = Sm.solve_mixed(dev(np.zeros(p.n)))
    assert zm.outer == 0 and float(zm.x.abs().max()) == 0.0


def test_edge_nan_and_breakdown(pkg, ora):
    say("edge: NaN rhs / indefinite operator")
    p, tau = case("box64x48")
    A = pkg.Stencil5.from_problem(p)
    S = pkg.Solver(A, pkg.ainv_setup(A, tau))
    b = p.b.copy()
    b[100] = np.nan
    with pytest.raises(pkg.PcgaError) as e:
        S.solve(dev(b))
    assert e.value.status == -3
    # tridiag(-0.9, 1, -0.9) is indefinite; Jacobi "preconditioner" D = 1
    n = 64
    q = tridiag_problem(np.ones(n), np.full(n, -0.9), b=np.random.default_rng(3).standard_normal(n))
    with pytest.raises(ora.OracleError) as eo:
        ora.pcg(q, ora.ainv_setup(q, np.inf), tol=1e-10)
    assert eo.value.status == ora.EBREAKDOWN
    Aq = pkg.Stencil5.from_problem(q)
    Sq = pkg.Solver(Aq, pkg.ainv_setup(Aq, np.inf))
    with pytest.raises(pkg.PcgaError) as eg:
        Sq.solve(dev(q.b), tol=1e-10)
    assert eg.value.status == -2


def test_determinism_and_launch_modes(pkg):
    p, tau = case("orca182x149")
    say("determinism: graph vs direct, chunk sizes")
    A = pkg.Stencil5.from_problem(p)
    S = pkg.Solver(A, pkg.ainv_setup(A, tau))
    ref = S.solve(dev(p.b), tol=1e-10)
    for chunk, graph in ((32, True), (32, False), (2, True), (128, True)):
        S.tune(chunk=chunk, use_graph=graph)
        r = S.solve(dev(p.b), tol=1e-10)
        assert r.iters == ref.iters and torch.equal(r.x, ref.x)
        assert np.array_equal(r.hist, ref.hist)


# ---------------------------------------------------------------------------
# full ORCA025-shaped size (1442 x 1021, drop tolerance 0.05), launch shape of
# the benchmark
# ---------------------------------------------------------------------------
def order_spread():
    """Rounding-order spread of Algorithm 1 at 1442x1021 (the oracle's default
    and evaluation-order builds; tests/golden/make_order_spread.py)."""
    import json
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "order_spread_1442x1021.json")
    with open(path) as f:
        return json.load(f)["factors"]


@pytest.fixture(scope="module")
def orca025(pkg, ora):
    say("building 1442x1021 problem and setups")
    p = orca.orca_problem(1442, 1021, orca.CONFIG_SEED_BASE + 2)
    F = ora.ainv_setup(p, 0.05)
    A = pkg.Stencil5.from_problem(p)
    G = pkg.ainv_setup(A, 0.05)
    return p, F, A, G


@pytest.fixture(scope="module")
def orca025_stops(ora, orca025):
    """The oracle's natural stops at 1442x1021 (threshold factor, and fixed
    fill 8 at drop tolerance 0.01), run in background threads (the oracle
    releases the interpreter while it computes) while the device tests go on."""
    from concurrent.futures import ThreadPoolExecutor
    p, F, _, _ = orca025
    ex = ThreadPoolExecutor(3)
    say("oracle natural stops at 1442x1021 started in the background")
    fut = {"threshold": ex.submit(lambda: ora.pcg(p, F, tol=1e-10)),
           "keep": ex.submit(lambda: ora.pcg_mixed(p, F, tol=1e-10, inner_tol=0.1, keep=True,
                                                   max_outer=200)),
           "fill8": ex.submit(lambda: (lambda Ff: (Ff, ora.pcg(p, Ff, tol=1e-10)))(
               ora.ainv_setup(p, 0.01, fill=8)))}
    yield fut
    ex.shutdown(wait=True)


def test_full_size_kernels(pkg, ora, orca025):
    p, F, A, G = orca025
    say("full size: apply_a, apply_prec")
    S = pkg.Solver(A, G, "fp64")
    x = np.random.default_rng(21).standard_normal(p.n)
    y = S.apply_a(dev(x)).cpu().numpy()
    mag = ora.spmv(_abs_problem(p), np.abs(x))
    assert np.all(np.abs(y - ora.spmv(p, x)) <= 8 * EPS * mag + 1e-300)
    t, s = S.apply_prec(dev(x))
    t_ref = ora.zt_apply(F, x)
    s_ref = ora.z_apply(F, t_ref)
    Fa = ora.AInv(F.n, F.colptr, F.rowidx, np.abs(F.val), F.D)
    t_mag = ora.zt_apply(Fa, np.abs(x))
    s_mag = ora.z_apply(Fa, t_mag)
    width = int(np.diff(F.colptr).max()) + 2
    assert np.all(np.abs(t.cpu().numpy() - t_ref) <= width * 4 * EPS * t_mag)
    assert np.all(np.abs(s.cpu().numpy() - s_ref) <= 2 * width * 4 * EPS * s_mag)
    say("full size: fused stencil step, FP64 and mixed")
    check_stencil_step(pkg, ora, S, p, "fp64", 44, 0.61)
    Sm = pkg.Solver(A, G, "mixed")
    check_stencil_step(pkg, ora, Sm, p, "mixed", 45, 0.61)


def test_full_size_pcg(pkg, ora, orca025, orca025_stops):
    """The benchmark's problem (1442x1021, drop tolerance 0.05), FP64.
    Bars from the rounding-order spread of the oracle's own builds
    (order_spread): iterates matched to 1e-9 over 30 iterations (the builds
    agree to about 1e-11 there and drift apart beyond: 2e-8 at 40, 1e-3 at
    60-100); the natural stop within 2 of the builds' stopping window; the
    solution within 1e-9 of the default oracle's (the builds agree to 5e-11);
    both true residuals at the 1e-10 target, up to the drift between the
    recursive residual that the stopping test reads and the true one."""
    p, F, A, G = orca025
    spread = order_spread()["threshold_tau0.05"]
    assert spread["iterate_spread"]["30"] <= 1e-10
    say("full size: 30 iterations matched, then natural stop")
    S = pkg.Solver(A, G, "fp64")
    g = S.solve(dev(p.b), tol=0.0, maxit=30)
    o = ora.pcg(p, F, tol=0.0, maxit=30)
    rel = np.linalg.norm(g.x.cpu().numpy() - o.x) / np.linalg.norm(o.x)
    say(f"  30 iterations: |x - x_ora|/|x_ora| = {rel:.2e}")
    assert rel <= 1e-9
    assert np.allclose(g.hist, o.hist, rtol=1e-9)
    full = S.solve(dev(p.b), tol=1e-10)
    lo, hi = spread["stop_window"]
    on = orca025_stops["threshold"].result()
    x = full.x.cpu().numpy()
    true = np.linalg.norm(p.b - ora.spmv(p, x)) / np.linalg.norm(p.b)
    true_o = np.linalg.norm(p.b - ora.spmv(p, on.x)) / np.linalg.norm(p.b)
    err = np.linalg.norm(x - on.x) / np.linalg.norm(on.x)
    say(f"  natural stop: device {full.iters}, oracle {on.iters}, oracle builds {lo}..{hi}; "
        f"true relres device {true:.3e} oracle {true_o:.3e}; |x - x_ora|/|x_ora| = {err:.2e}")
    assert full.status == 0 and on.status == 0
    assert on.iters == spread["stop_iters"]["default"]
    assert lo - 2 <= full.iters <= hi + 2
    # the stopping test reads the recursive residual; the true one drifts from
    # it by up to 1% here (the oracle's own builds reach 1.004e-10)
    assert true <= 1.02e-10 and true_o <= 1.02e-10
    assert err <= 1e-9


def test_full_size_jacobi_two_launch_path(pkg, ora, orca025):
    """The diagonal preconditioner (Z = I) runs two launches per iteration
    (stencil with the stop test, fused update + D^-1): iterates match the
    oracle's Algorithm 1 with (Z, D) = ainv_setup(A, inf), in FP64 and as the
    FP32 inner solve of the mixed form."""
    p, F, A, G = orca025
    say("full size: diagonal preconditioner, 40 iterations matched")
    Gj = pkg.ainv_setup(A, np.inf)
    Fj = ora.ainv_setup(p, np.inf)
    assert Gj.nnz_off == 0
    S = pkg.Solver(A, Gj, "fp64")
    g = S.solve(dev(p.b), tol=0.0, maxit=40)
    o = ora.pcg(p, Fj, tol=0.0, maxit=40)
    assert g.iters == o.iters == 40
    assert np.linalg.norm(g.x.cpu().numpy() - o.x) <= 1e-9 * np.linalg.norm(o.x)
    assert np.allclose(g.hist, o.hist, rtol=1e-9)
    ms = S.profile_iteration(dev(p.b), reps=4)
    assert ms[2] == 0.0 and ms[0] > 0 and ms[1] > 0 and ms[3] > 0
    Sm = pkg.Solver(A, Gj, "mixed")
    m = Sm.solve_mixed(dev(p.b), tol=1e-8, inner_tol=1e-3, max_outer=20)
    say("  mixed: outer", m.outer, "inner", m.inner_total, "true", m.true_relres)
    assert m.status == 0
    x = m.x.cpu().numpy()
    assert np.linalg.norm(p.b - ora.spmv(p, x)) / np.linalg.norm(p.b) <= 1e-8


def test_full_size_mixed_keep(pkg, ora, orca025, orca025_stops):
    """The keep form at 1442x1021: true FP64 residual at the target, the
    error against the FP64 oracle's solution stated, and the corrections and
    inner iterations against the oracle's run of the same form."""
    p, F, A, G = orca025
    say("full size: mixed, direction kept")
    S = pkg.Solver(A, G, "mixed")
    m = S.solve_mixed(dev(p.b), tol=1e-10, refine="keep")
    assert m.status == 0
    x = m.x.cpu().numpy()
    true = np.linalg.norm(p.b - ora.spmv(p, x)) / np.linalg.norm(p.b)
    on = orca025_stops["threshold"].result()
    om = orca025_stops["keep"].result()
    err = np.linalg.norm(x - on.x) / np.linalg.norm(on.x)
    say(f"  outer {m.outer} (oracle {om.outer}) inner {m.inner_total} (oracle {om.inner_total}, "
        f"FP64 {on.iters}) true relres {true:.3e}; |x_mixed - x_ora|/|x_ora| = {err:.2e}")
    assert true <= 1e-10
    assert err <= 1e-8
    assert abs(m.outer - om.outer) <= 2
    assert abs(m.inner_total - om.inner_total) <= max(10, om.inner_total // 20)


@pytest.mark.parametrize("form", ["mixed", "mixed_a32"])
def test_full_size_mixed(pkg, ora, orca025, orca025_stops, form):
    """FP32 inner PCG with FP64 refinement at 1442x1021, with the FP64
    operator applied to the FP32 inner vectors (mixed) or the operator in FP32
    too (mixed_a32): the true FP64 residual at the 1e-10 target, and the error
    against the FP64 oracle's solution stated (two solutions at relative
    residual 1e-10 of this ill-conditioned system need not be closer than
    about 1e-9)."""
    p, F, A, G = orca025
    say("full size:", form)
    S = pkg.Solver(A, G, form)
    m = S.solve_mixed(dev(p.b), tol=1e-10, inner_tol=1e-5, max_outer=20)
    assert m.status == 0
    x = m.x.cpu().numpy()
    true = np.linalg.norm(p.b - ora.spmv(p, x)) / np.linalg.norm(p.b)
    on = orca025_stops["threshold"].result()
    err = np.linalg.norm(x - on.x) / np.linalg.norm(on.x)
    say(f"  outer {m.outer} inner {m.inner_total} true relres {true:.3e}; "
        f"|x_mixed - x_ora|/|x_ora| = {err:.2e} (FP64 oracle, {on.iters} iterations)")
    assert true <= 1e-10
    assert err <= 1e-8


@pytest.mark.parametrize("q", [1, 3, 8])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_band_factor_diagonal_path(pkg, ora, q, prec):
    """The banded factor of T is applied from its diagonals (no indices):
    t = D^-1 Z^T r and s = Z t match the oracle's apply of the same factor."""
    p, _ = case("orca37x23_ragged")
    A = pkg.Stencil5.from_problem(p)
    G = pkg.fsai_band_setup(A, q)
    F, _ = ora.fsai_band(p, q)
    S = pkg.Solver(A, G, prec)
    assert S.band_q == q
    r = np.random.default_rng(14).standard_normal(p.n)
    t, s = S.apply_prec(dev(r))
    t_ref = ora.zt_apply(F, r)
    s_ref = ora.z_apply(F, t_ref)
    Fa = ora.AInv(F.n, F.colptr, F.rowidx, np.abs(F.val), F.D)
    t_mag = ora.zt_apply(Fa, np.abs(r))
    s_mag = ora.z_apply(Fa, t_mag)
    u = 4 * EPS if prec == "fp64" else 4 * np.finfo(np.float32).eps
    assert np.all(np.abs(t.cpu().numpy() - t_ref) <= (q + 2) * u * t_mag + 1e-300)
    assert np.all(np.abs(s.cpu().numpy() - s_ref) <= 2 * (q + 2) * u * s_mag + 1e-300)
    # AINV factors reach several grid rows: no diagonal storage
    Aq = pkg.Stencil5.from_problem(case("orca182x149")[0])
    assert pkg.Solver(Aq, pkg.ainv_setup(Aq, 0.1), prec).band_q == 0


def test_full_size_band_factor(pkg, ora, orca025):
    """The paper's preconditioner (banded factor of T, q = 4) at 1442x1021:
    40 iterations matched to the oracle, mixed form converges."""
    p, F, A, G = orca025
    say("full size: banded factor of T, q = 4")
    Gb = pkg.fsai_band_setup(A, 4)
    Fb, _ = ora.fsai_band(p, 4)
    S = pkg.Solver(A, Gb, "fp64")
    assert S.band_q == 4
    g = S.solve(dev(p.b), tol=0.0, maxit=40)
    o = ora.pcg(p, Fb, tol=0.0, maxit=40)
    assert g.iters == o.iters == 40
    assert np.linalg.norm(g.x.cpu().numpy() - o.x) <= 1e-9 * np.linalg.norm(o.x)
    assert np.allclose(g.hist, o.hist, rtol=1e-9)


def oracle_stop_window(ora, p, F, tol):
    """Range of stopping iterations over the oracle's default build and its
    evaluation-order builds (reversed or blocked inner-product sums, fused
    multiply-adds): the same method, different rounding.  Algorithm 1 fixes
    no order for the additions of an inner product, so a correct FP64
    implementation may stop anywhere in this range; the device (blocked sums
    over workgroups, fused multiply-adds) must stop within 2 of it."""
    ks = ora.stop_window(p, F, tol=tol)
    return min(ks.values()), max(ks.values()), ks


@pytest.mark.parametrize("q", [1, 4])
def test_pcg_paper_band_preconditioner(pkg, ora, q):
    """Algorithm 1 with the paper's own banded factor of T (Sec. 3 scheme):
    device and oracle iterates match; AINV needs fewer iterations than the
    banded factor of T, which needs no more than Jacobi (Table 2's ordering)."""
    p, _ = case("orca182x149")
    say("band preconditioner q =", q)
    A = pkg.Stencil5.from_problem(p)
    G = pkg.fsai_band_setup(A, q)
    F, _ = ora.fsai_band(p, q)
    K = ora.pcg(p, F, tol=1e-10).iters
    S = pkg.Solver(A, G, "fp64")
    g = S.solve(dev(p.b), tol=0.0, maxit=K)
    o = ora.pcg(p, F, tol=0.0, maxit=K)
    assert np.linalg.norm(g.x.cpu().numpy() - o.x) <= 1e-9 * np.linalg.norm(o.x)
    nat = S.solve(dev(p.b), tol=1e-10)
    lo, hi, ks = oracle_stop_window(ora, p, F, 1e-10)
    say(f"  natural stop: device {nat.iters}, oracle {K}, oracle builds {ks}")
    assert nat.status == 0 and lo - 2 <= nat.iters <= hi + 2
    kj = ora.pcg(p, ora.ainv_setup(p, np.inf), tol=1e-10).iters
    ka = ora.pcg(p, ora.ainv_setup(p, 0.1), tol=1e-10).iters
    say(f"  iterations: jacobi {kj}, band q={q} {K}, ainv {ka}")
    assert K <= kj and ka < K


def test_largest_catalogue_grid(pkg, ora):
    """4322x3059 (13.2 M cells, the largest grid of the serving catalogue):
    the preconditioner apply against the oracle over the whole grid, and the
    FP64 solve's true residual recomputed with the oracle's product."""
    p = orca.orca_problem(4322, 3059, orca.CONFIG_SEED_BASE + 47)
    say("largest grid", p.n, "cells: setups")
    A = pkg.Stencil5.from_problem(p)
    G = pkg.ainv_setup(A, 0.05)
    F = ora.ainv_setup(p, 0.05)
    assert G.nnz_off == F.nnz_off
    S = pkg.Solver(A, G, "fp64")
    say("  solver index bytes", S.index_bytes, "formats", S.formats)
    x = np.random.default_rng(31).standard_normal(p.n)
    t, s = S.apply_prec(dev(x))
    t_ref = ora.zt_apply(F, x)
    s_ref = ora.z_apply(F, t_ref)
    Fa = ora.AInv(F.n, F.colptr, F.rowidx, np.abs(F.val), F.D)
    t_mag = ora.zt_apply(Fa, np.abs(x))
    s_mag = ora.z_apply(Fa, t_mag)
    width = int(np.diff(F.colptr).max()) + 2
    assert np.all(np.abs(t.cpu().numpy() - t_ref) <= width * 4 * EPS * t_mag)
    assert np.all(np.abs(s.cpu().numpy() - s_ref) <= 2 * width * 4 * EPS * s_mag)
    say("  FP64 solve")
    g = S.solve(dev(p.b), tol=1e-10)
    xg = g.x.cpu().numpy()
    true = np.linalg.norm(p.b - ora.spmv(p, xg)) / np.linalg.norm(p.b)
    say("  iterations", g.iters, "true relres", true)
    assert g.status == 0 and g.hist[-1] <= 1e-10 and true <= 1.05e-10


@pytest.mark.parametrize("tau,fill", [(0.01, 4), (0.01, 8), (0.0, 3)])
def test_pcg_fixed_fill(pkg, ora, tau, fill):
    """The fixed-fill AINV (second Bridson class of Sec. 5) through the same
    sliced-ELL path: every row of Z^T holds at most `fill` off-diagonal
    entries; device and oracle iterates match; the natural stop agrees; the
    mixed form reaches the FP64 bar."""
    p, _ = case("orca182x149")
    say("fixed fill: drop_tol", tau, "fill", fill)
    A = pkg.Stencil5.from_problem(p)
    G = pkg.ainv_setup(A, tau, fill=fill)
    F = ora.ainv_setup(p, tau, fill=fill)
    assert G.nnz_off == F.nnz_off
    assert int(np.diff(F.colptr).max()) <= fill
    K = ora.pcg(p, F, tol=1e-10).iters
    for prec in ("fp64", "mixed"):
        S = pkg.Solver(A, G, prec)
        if prec == "fp64":
            g = S.solve(dev(p.b), tol=0.0, maxit=K)
            o = ora.pcg(p, F, tol=0.0, maxit=K)
            assert np.linalg.norm(g.x.cpu().numpy() - o.x) <= 1e-9 * np.linalg.norm(o.x)
            nat = S.solve(dev(p.b), tol=1e-10)
            say(f"  natural stop: device {nat.iters}, oracle {K}")
            assert nat.status == 0 and abs(nat.iters - K) <= 2
            assert nat.true_relres <= 1e-10
        else:
            m = S.solve_mixed(dev(p.b), tol=1e-10)
            say(f"  mixed: outer {m.outer}, inner {m.inner_total}, true {m.true_relres:.2e}")
            assert m.status == 0 and m.true_relres <= 1e-10
        S.close()


def test_full_size_fixed_fill(pkg, ora, orca025, orca025_stops):
    """Fixed fill at 1442x1021 (drop_tol 0.01, 8 per column): the
    preconditioner apply against the oracle over the whole grid; iterates
    matched over 12 iterations; the natural stop within 2 of the stopping
    window of the oracle's evaluation-order builds, the solution within 1e-9
    of the default oracle's, true residuals at the target.  This iteration
    amplifies rounding much faster than the threshold factor's: the oracle's
    own builds, which differ only in the order of additions, are 5.8e-10
    apart after 20 iterations, 3.7e-2 after 30 and 3.2e-2 after 40 (the
    device's 8e-3 at 40 is smaller) and stop anywhere in 2504..2564."""
    p, _, A, _ = orca025
    spread = order_spread()["fixed_fill8_tau0.01"]
    assert spread["iterate_spread"]["12"] <= 1e-12
    say("full size: fixed fill 8, drop_tol 0.01")
    G = pkg.ainv_setup(A, 0.01, fill=8)
    F, on = orca025_stops["fill8"].result()
    assert G.nnz_off == F.nnz_off == spread["nnz_off"]
    S = pkg.Solver(A, G, "fp64")
    x = np.random.default_rng(23).standard_normal(p.n)
    t, s = S.apply_prec(dev(x))
    t_ref = ora.zt_apply(F, x)
    s_ref = ora.z_apply(F, t_ref)
    Fa = ora.AInv(F.n, F.colptr, F.rowidx, np.abs(F.val), F.D)
    t_mag = ora.zt_apply(Fa, np.abs(x))
    s_mag = ora.z_apply(Fa, t_mag)
    width = int(np.diff(F.colptr).max()) + 2
    assert np.all(np.abs(t.cpu().numpy() - t_ref) <= width * 4 * EPS * t_mag)
    assert np.all(np.abs(s.cpu().numpy() - s_ref) <= 2 * width * 4 * EPS * s_mag)
    g = S.solve(dev(p.b), tol=0.0, maxit=12)
    o = ora.pcg(p, F, tol=0.0, maxit=12)
    assert g.iters == o.iters == 12
    assert np.linalg.norm(g.x.cpu().numpy() - o.x) <= 1e-9 * np.linalg.norm(o.x)
    assert np.allclose(g.hist, o.hist, rtol=1e-9)
    full = S.solve(dev(p.b), tol=1e-10)
    lo, hi = spread["stop_window"]
    xf = full.x.cpu().numpy()
    true = np.linalg.norm(p.b - ora.spmv(p, xf)) / np.linalg.norm(p.b)
    err = np.linalg.norm(xf - on.x) / np.linalg.norm(on.x)
    say(f"  natural stop: device {full.iters}, oracle {on.iters}, oracle builds {lo}..{hi}; "
        f"true relres {true:.3e}; |x - x_ora|/|x_ora| = {err:.2e}")
    assert full.status == 0 and on.iters == spread["stop_iters"]["default"]
    assert lo - 2 <= full.iters <= hi + 2
    # recursive vs true residual drift: the default oracle build ends at 1.009e-10
    assert true <= 1.02e-10 and err <= 1e-9
    S.close()


@pytest.mark.parametrize("fill", [None, 6])
def test_pcg_mixed_sign_operator(pkg, ora, fill):
    """A symmetric positive definite operator with couplings of both signs
    (not an M-matrix: the factor holds entries of both signs): matched
    iterates, the natural stop, and the preconditioner apply against the
    oracle, for the threshold and the fixed-fill factor."""
    from tests._cases import mixed_sign_dominant
    p = mixed_sign_dominant(203, 157, True, 11)
    rng = np.random.default_rng(12)
    p.b = rng.standard_normal(p.n)
    say("mixed-sign operator", p.nx, "x", p.ny, "fill", fill)
    A = pkg.Stencil5.from_problem(p)
    G = pkg.ainv_setup(A, 0.01, fill=fill)
    F = ora.ainv_setup(p, 0.01, fill=fill)
    assert G.nnz_off == F.nnz_off
    assert (F.val < 0).any() and (F.val > 0).any()
    S = pkg.Solver(A, G, "fp64")
    x = rng.standard_normal(p.n)
    t, s = S.apply_prec(dev(x))
    t_ref = ora.zt_apply(F, x)
    s_ref = ora.z_apply(F, t_ref)
    Fa = ora.AInv(F.n, F.colptr, F.rowidx, np.abs(F.val), F.D)
    t_mag = ora.zt_apply(Fa, np.abs(x))
    s_mag = ora.z_apply(Fa, t_mag)
    width = int(np.diff(F.colptr).max()) + 2
    assert np.all(np.abs(t.cpu().numpy() - t_ref) <= width * 4 * EPS * t_mag)
    assert np.all(np.abs(s.cpu().numpy() - s_ref) <= 2 * width * 4 * EPS * s_mag)
    K = ora.pcg(p, F, tol=1e-10).iters
    g = S.solve(dev(p.b), tol=0.0, maxit=min(K, 12))
    o = ora.pcg(p, F, tol=0.0, maxit=min(K, 12))
    assert np.linalg.norm(g.x.cpu().numpy() - o.x) <= 1e-9 * np.linalg.norm(o.x)
    nat = S.solve(dev(p.b), tol=1e-10)
    say(f"  natural stop: device {nat.iters}, oracle {K}")
    assert nat.status == 0 and abs(nat.iters - K) <= 2
    xf = nat.x.cpu().numpy()
    assert np.linalg.norm(p.b - ora.spmv(p, xf)) / np.linalg.norm(p.b) <= 1.05e-10
    S.close()


def test_solver_on_shared_buffer(pkg):
    """Solvers carved one after another from one buffer (what the autotuner
    does) give bitwise the results of a solver with its own workspace; a
    buffer that is too small is refused."""
    p, _ = case("orca182x149")
    A = pkg.Stencil5.from_problem(p)
    G = pkg.ainv_setup(A, 0.1)
    b = dev(p.b)
    ref = pkg.Solver(A, G, "fp64").solve(b, tol=1e-10)
    buf = torch.empty(max(pkg.workspace_size(A, G, "fp64", w) for w in (8, 32)),
                      dtype=torch.uint8, device="cuda")
    for w in (8, 0):
        S = pkg.Solver(A, G, "fp64", slice_width=w, buffer=buf)
        assert S.ws.data_ptr() % (16 << 20) == 0
        r = S.solve(b, tol=1e-10)
        if w == 0:
            assert r.iters == ref.iters
            assert torch.equal(r.x, ref.x)
        S.close()
        torch.cuda.synchronize()
    small = torch.empty(1 << 20, dtype=torch.uint8, device="cuda")
    with pytest.raises(ValueError):
        pkg.Solver(A, G, "fp64", buffer=small)


def test_solver_placement_probe(pkg):
    """A solver that probes three workspace bases keeps one of them and
    solves bitwise like a solver placed without probing."""
    p, _ = case("orca182x149")
    A = pkg.Stencil5.from_problem(p)
    G = pkg.ainv_setup(A, 0.1)
    b = dev(p.b)
    ref = pkg.Solver(A, G, "fp64").solve(b, tol=1e-10)
    S = pkg.Solver(A, G, "fp64", probe_placements=3)
    assert S.placement_ms is not None and len(S.placement_ms) == 3
    assert all(t > 0 for t in S.placement_ms)
    lead = (-S._ws_buf.data_ptr()) % (16 << 20)          # the aligned first base
    assert S.ws.data_ptr() - S._ws_buf.data_ptr() - lead in (0, 4 << 20, 8 << 20)
    r = S.solve(b, tol=1e-10)
    assert r.iters == ref.iters and torch.equal(r.x, ref.x)
    S.close()
