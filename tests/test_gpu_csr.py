"""General sparse (CSR) operator on the device vs the FP64 oracle (needs an MI355X).

A CSR matrix is laid out in the sliced ELL of Z (its diagonal among the
entries); the iteration's first kernel recomputes d = s + beta d at every row
it gathers while it forms q = A d.  Bars as for the grid: the operator
product within a few ulp of the oracle's (scaled by the magnitude of its
terms), iterates matched to 1e-9 while the oracle's own evaluation-order
builds agree, the natural stop within 2 of their stopping window, solutions
within 1e-9 of the oracle's, true residuals at the target.
"""
import sys

import numpy as np
import pytest

from gen import orca
from gen.unstructured import csr_from_grid, unstructured_problem

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

EPS = np.finfo(np.float64).eps


def say(*a):
    print("[gpu-csr]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def pkg():
    if not torch.cuda.is_available():
        pytest.skip("no ROCm device")
    import paper_1210_1878_amd as P
    return P


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


CASES = {
    "unstructured3k_laplacian": (lambda: unstructured_problem(3000, 41), 0.05),
    "unstructured3k_mixed": (lambda: unstructured_problem(3000, 42, kind="mixed"), 0.02),
    "unstructured40k_laplacian": (lambda: unstructured_problem(40000, 43), 0.05),
    "unstructured777_ragged": (lambda: unstructured_problem(777, 44, k=9), 0.1),
    "grid182x149_as_csr": (lambda: csr_from_grid(orca.orca_problem(182, 149, orca.CONFIG_SEED_BASE + 1)), 0.1),
    "unstructured5k_jacobi": (lambda: unstructured_problem(5000, 45), np.inf),
}

_cache = {}


def case(name):
    if name not in _cache:
        mk, tau = CASES[name]
        _cache[name] = (mk(), tau)
    return _cache[name]


def _abs(p):
    import copy
    q = copy.copy(p)
    q.val = np.abs(p.val)
    return q


@pytest.mark.parametrize("name", list(CASES))
def test_csr_apply_a_and_prec(pkg, ora, name):
    p, tau = case(name)
    say("apply", name, p.n, "nnz", p.nnz)
    A = pkg.CsrMatrix.from_problem(p)
    G = pkg.ainv_setup(A, tau)
    S = pkg.Solver(A, G, "fp64")
    x = np.random.default_rng(12).standard_normal(p.n)
    y = S.apply_a(dev(x)).cpu().numpy()
    mag = ora.spmv(_abs(p), np.abs(x))
    maxrow = int(np.diff(p.rowptr).max())
    assert np.all(np.abs(y - ora.spmv(p, x)) <= (maxrow + 2) * EPS * mag)
    F = ora.ainv_setup(p, tau)
    t, s = S.apply_prec(dev(x))
    t_ref = ora.zt_apply(F, x)
    s_ref = ora.z_apply(F, t_ref)
    Fa = ora.AInv(F.n, F.colptr, F.rowidx, np.abs(F.val), F.D)
    t_mag = ora.zt_apply(Fa, np.abs(x))
    s_mag = ora.z_apply(Fa, t_mag)
    width = (int(np.diff(F.colptr).max()) if F.nnz_off else 0) + 2
    assert np.all(np.abs(t.cpu().numpy() - t_ref) <= width * 4 * EPS * t_mag)
    assert np.all(np.abs(s.cpu().numpy() - s_ref) <= 2 * width * 4 * EPS * s_mag)


@pytest.mark.parametrize("name", list(CASES))
def test_csr_pcg_matched_and_natural_stop(pkg, ora, name):
    p, tau = case(name)
    A = pkg.CsrMatrix.from_problem(p)
    G = pkg.ainv_setup(A, tau)
    F = ora.ainv_setup(p, tau)
    assert G.nnz_off == F.nnz_off
    S = pkg.Solver(A, G, "fp64")
    K = 12
    g = S.solve(dev(p.b), tol=0.0, maxit=K)
    o = ora.pcg(p, F, tol=0.0, maxit=K)
    rel = np.linalg.norm(g.x.cpu().numpy() - o.x) / np.linalg.norm(o.x)
    assert g.iters == o.iters == K
    assert rel <= 1e-9 and np.allclose(g.hist, o.hist, rtol=1e-9)
    nat = S.solve(dev(p.b), tol=1e-10)
    ks = ora.stop_window(p, F, tol=1e-10)
    on = ora.pcg(p, F, tol=1e-10)
    x = nat.x.cpu().numpy()
    true = np.linalg.norm(p.b - ora.spmv(p, x)) / np.linalg.norm(p.b)
    err = np.linalg.norm(x - on.x) / np.linalg.norm(on.x)
    say(f"{name}: {K} iterations matched to {rel:.1e}; natural stop device {nat.iters}, "
        f"oracle builds {sorted(set(ks.values()))}; true relres {true:.2e}; "
        f"|x - x_ora|/|x_ora| {err:.1e}")
    assert nat.status == 0
    assert min(ks.values()) - 2 <= nat.iters <= max(ks.values()) + 2
    assert true <= 1.02e-10 and abs(true - nat.true_relres) <= 1e-3 * true + 1e-13
    assert err <= 1e-9


def test_csr_grid_operator_matches_five_point_path(pkg, ora):
    """The same grid operator through the five-point kernels and through the
    CSR kernels: iterates matched to 1e-9 over 30 iterations, equal natural
    stops within the oracle builds' window."""
    p = orca.orca_problem(182, 149, orca.CONFIG_SEED_BASE + 1)
    C = csr_from_grid(p)
    A5, Ac = pkg.Stencil5.from_problem(p), pkg.CsrMatrix.from_problem(C)
    G5, Gc = pkg.ainv_setup(A5, 0.1), pkg.ainv_setup(Ac, 0.1)
    S5, Sc = pkg.Solver(A5, G5, "fp64"), pkg.Solver(Ac, Gc, "fp64")
    a = S5.solve(dev(p.b), tol=0.0, maxit=30).x.cpu().numpy()
    c = Sc.solve(dev(p.b), tol=0.0, maxit=30).x.cpu().numpy()
    assert np.linalg.norm(a - c) <= 1e-9 * np.linalg.norm(a)
    n5, nc = S5.solve(dev(p.b), tol=1e-10), Sc.solve(dev(p.b), tol=1e-10)
    ks = ora.stop_window(p, ora.ainv_setup(p, 0.1), tol=1e-10)
    say("grid as CSR: stops five-point", n5.iters, "csr", nc.iters, "oracle builds", ks)
    for it in (n5.iters, nc.iters):
        assert min(ks.values()) - 2 <= it <= max(ks.values()) + 2


def test_csr_edges_and_noalloc(pkg, ora):
    p, tau = case("unstructured3k_mixed")
    A = pkg.CsrMatrix.from_problem(p)
    S = pkg.Solver(A, pkg.ainv_setup(A, tau), "fp64")
    z = S.solve(dev(np.zeros(p.n)), tol=1e-10)
    assert z.iters == 0 and z.status == 0 and float(z.x.abs().max()) == 0.0
    ref = S.solve(dev(p.b), tol=1e-10)
    x = torch.zeros(p.n, dtype=torch.float64, device="cuda")
    na = S.solve_noalloc(dev(p.b), x, tol=1e-10)
    assert na.iters == ref.iters and torch.equal(x, ref.x)
    # warm start from the solution: converged at once
    w = S.solve(dev(p.b), x0=ref.x, tol=1e-9)
    assert w.iters <= 2
    # five-point-only calls are refused on a CSR solver
    from paper_1210_1878_amd import _lib
    with pytest.raises(_lib.PcgaError):
        S.step_stencil(dev(p.b), dev(p.b), 0.5)
