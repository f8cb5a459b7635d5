"""The time step around the solve on the device vs the oracle (needs an MI355X):
the right-hand side of eq. (8), the sea-surface update of eq. (1) and the
first guess of Algorithm 1 bitwise (the same FP64 operations in the same
order, no contraction), then whole time steps (right-hand side, first guess,
FP64 solve, sea-surface update) to the solve's bar."""
import sys

import numpy as np
import pytest

from gen import orca

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-timestep]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def pkg():
    if not torch.cuda.is_available():
        pytest.skip("no ROCm device")
    import paper_1210_1878_amd as P
    return P


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _solver(P, p, tau=0.1):
    A = P.Stencil5.from_problem(p)
    return P.Solver(A, P.ainv_setup(A, tau), "fp64")


GRIDS = {
    "orca182x149": lambda: orca.orca_problem(182, 149, orca.CONFIG_SEED_BASE + 1),
    "orca37x23_ragged": lambda: orca.orca_problem(37, 23, 5),
    "orca1442x1021": lambda: orca.orca_problem(1442, 1021, orca.CONFIG_SEED_BASE + 2),
    "box64x48_closed": lambda: orca.box_problem(),
}


@pytest.mark.parametrize("name", list(GRIDS))
def test_rhs_bitwise(pkg, ora, name):
    p = GRIDS[name]()
    say(name, "n", p.n, "periodic", p.periodic)
    S = _solver(pkg, p, 0.1 if p.n < 10**6 else 0.05)
    if name.startswith("box"):
        rng = np.random.default_rng(4)
        faces = [rng.uniform(0.5, 2.0, p.n), rng.standard_normal(p.n),
                 rng.uniform(0.5, 2.0, p.n), rng.standard_normal(p.n)]
    else:
        faces = list(orca.orca_transports(p, 5, seed=9))
    b = S.ts_rhs(*[_dev(f) for f in faces])
    torch.cuda.synchronize()
    want = ora.ts_rhs(p.nx, p.ny, p.periodic, *faces)
    got = b.cpu().numpy()
    assert np.array_equal(got, want), f"max |diff| {np.abs(got - want).max()}"


def test_eta_and_guess_bitwise(pkg, ora):
    p = GRIDS["orca37x23_ragged"]()
    S = _solver(pkg, p)
    rng = np.random.default_rng(7)
    e, d1, d2 = (rng.standard_normal(p.n) for _ in range(3))
    got = S.ts_eta(_dev(e), _dev(d1), 0.37).cpu().numpy()
    assert np.array_equal(got, ora.ts_eta(e, d1, 0.37))
    for a, c in ((2.0, -1.0), (1.0, 0.0), (2.0, 0.0), (1.7, -0.3)):
        g = S.ts_guess(_dev(d1), _dev(d2) if c else None, a, c).cpu().numpy()
        assert np.array_equal(g, ora.ts_guess(d1, d2, a, c)), (a, c)


def test_errors(pkg):
    p = GRIDS["orca37x23_ragged"]()
    S = _solver(pkg, p)
    x = _dev(np.zeros(p.n))
    with pytest.raises(Exception):
        S.ts_eta(x, x, -1.0)
    with pytest.raises(ValueError):
        S.ts_guess(x, None, 2.0, -1.0)


@pytest.mark.parametrize("guess", [(1.0, 0.0), (2.0, -1.0)])
def test_time_steps_match_oracle(pkg, ora, guess):
    """Four time steps on 182x149: right-hand side from the transports of the
    step, first guess from the previous solutions, FP64 solve to 1e-10,
    sea-surface update; the device path and the oracle run the same steps."""
    p = GRIDS["orca182x149"]()
    tau, dt, tol = 0.1, 0.5, 1e-10
    S = _solver(pkg, p, tau)
    F = ora.ainv_setup(p, tau)
    a, c = guess
    n = p.n
    eta_d = [_dev(np.zeros(n)), _dev(np.zeros(n))]      # eta^{n-1}, eta^n
    eta_o = [np.zeros(n), np.zeros(n)]
    Dd, Do = [], []
    for t in range(4):
        faces = orca.orca_transports(p, t, seed=21)
        bd = S.ts_rhs(*[_dev(f) for f in faces])
        bo = ora.ts_rhs(p.nx, p.ny, p.periodic, *faces)
        if t == 0:
            x0d, x0o = None, np.zeros(n)
        elif t == 1 or c == 0.0:
            x0d = S.ts_guess(Dd[-1], None, 1.0 if t == 1 else a, 0.0)
            x0o = ora.ts_guess(Do[-1], None, 1.0 if t == 1 else a, 0.0)
        else:
            x0d = S.ts_guess(Dd[-1], Dd[-2], a, c)
            x0o = ora.ts_guess(Do[-1], Do[-2], a, c)
        rd = S.solve(bd, x0d, tol=tol)
        ro = ora.pcg(p, F, b=bo, x0=x0o, tol=tol)
        say("step", t, "guess", guess, "iters gpu", rd.iters, "oracle", ro.iters)
        assert rd.status == 0 and ro.status == 0
        assert abs(rd.iters - ro.iters) <= 2
        xd = rd.x.cpu().numpy()
        assert np.linalg.norm(xd - ro.x) <= 1e-8 * np.linalg.norm(ro.x)
        Dd.append(rd.x)
        Do.append(ro.x)
        # eq. (1): eta^{n+1} = eta^{n-1} - 2 dt D^n
        eta_d = [eta_d[1], S.ts_eta(eta_d[0], rd.x, dt)]
        eta_o = [eta_o[1], ora.ts_eta(eta_o[0], ro.x, dt)]
    ed = eta_d[1].cpu().numpy()
    assert np.linalg.norm(ed - eta_o[1]) <= 1e-8 * np.linalg.norm(eta_o[1])
