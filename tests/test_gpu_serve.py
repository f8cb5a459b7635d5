"""Continuous-batching server (needs an MI355X): every served time step meets
the FP64 target, equals the same solve run alone, and admission respects the
device-memory budget."""
import sys

import numpy as np
import pytest

from gen import orca

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-serve]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def setup():
    if not torch.cuda.is_available():
        pytest.skip("no ROCm device")
    import paper_1210_1878_amd as P
    from paper_1210_1878_amd import serve
    probs = [orca.orca_problem(nx, ny, 100 + i) for i, (nx, ny) in
             enumerate([(60, 45), (91, 62), (37, 23)])]
    return P, serve, probs


@pytest.mark.parametrize("refine", ["keep", "restart"])
def test_served_steps_correct_and_equal_alone(setup, ora, refine):
    P, serve, probs = setup
    say("serving 12 time steps on 3 grids, refinement", refine)
    srv = serve.Server(probs, drop_tol=0.1, device="cuda", chunk=8, refine=refine)
    reqs = serve.poisson_arrivals(rate=400.0, count=12, n_grids=len(probs), seed=7)
    stepper = serve.TimeStepper(probs, torch.device("cuda"), seed=3)
    done = srv.run(reqs, make_rhs=stepper, on_done=stepper.done)
    assert len(done) == 12
    overlapped = 0
    for r in done:
        p = probs[r.grid]
        b = r.b.cpu().numpy()
        x = r.x.cpu().numpy()
        true = np.linalg.norm(b - ora.spmv(p, x)) / np.linalg.norm(b)
        assert r.status == 0 and true <= 1e-10
        # the same solve alone in a fresh batch gives bitwise the same x
        Bt = P.Batch(max_slots=2, chunk=8)
        s = Bt.add(srv.solvers[r.grid], r.b.unsqueeze(0), X0=r.x0.unsqueeze(0), tol=srv.tol,
                   inner_tol=srv.inner_tol, max_outer=srv.max_outer, refine=srv.refine)
        X, q = Bt.solve()[s]
        assert torch.equal(X[0], r.x)
        overlapped += any(o is not r and o.admitted < r.finished and o.finished > r.admitted
                          for o in done)
    stats = serve.latency_stats(done)
    say("  stats", stats, "overlapping requests", overlapped)
    assert overlapped > 0         # requests did share the device
    # warm starts: later steps of a grid need fewer inner iterations than its first
    firsts = {}
    for r in sorted(done, key=lambda r: r.arrival):
        firsts.setdefault(r.grid, r)
    later = [r for r in done if firsts[r.grid] is not r]
    assert later and np.mean([r.inner for r in later]) < np.mean([r.inner for r in firsts.values()])


def test_admission_by_footprint(setup):
    P, serve, probs = setup
    say("admission under a tight memory budget")
    srv = serve.Server(probs, drop_tol=0.1, device="cuda", chunk=8)
    srv.budget = max(srv.item_bytes)      # room for one request at a time
    reqs = serve.poisson_arrivals(rate=1000.0, count=6, n_grids=len(probs), seed=9)
    stepper = serve.TimeStepper(probs, torch.device("cuda"), seed=4)
    peak = [0]
    orig_admit = srv.admit

    def admit(req, now):
        s = orig_admit(req, now)
        peak[0] = max(peak[0], srv.in_flight_bytes)
        return s
    srv.admit = admit
    done = srv.run(reqs, make_rhs=stepper, on_done=stepper.done)
    assert len(done) == 6 and all(r.status == 0 for r in done)
    assert peak[0] <= srv.budget


def test_saturate_closed_loop(setup, ora):
    P, serve, probs = setup
    say("closed loop: every grid keeps one step in flight")
    srv = serve.Server(probs, drop_tol=0.1, device="cuda", chunk=8)
    stepper = serve.TimeStepper(probs, torch.device("cuda"), seed=5)
    done, el = srv.saturate(0.3, make_rhs=stepper, on_done=stepper.done)
    per = [sum(1 for r in done if r.grid == g) for g in range(len(probs))]
    say("  completions per grid", per, "in", round(el, 3), "s")
    assert all(c >= 1 for c in per)
    assert not srv.busy.count(True) and srv.in_flight_bytes == 0
    for r in done:
        p = probs[r.grid]
        b, x = r.b.cpu().numpy(), r.x.cpu().numpy()
        assert r.status == 0
        assert np.linalg.norm(b - ora.spmv(p, x)) / np.linalg.norm(b) <= 1e-10
    # steps of one grid never overlap
    for g in range(len(probs)):
        rs = sorted((r for r in done if r.grid == g), key=lambda r: r.admitted)
        assert all(a.finished <= b.admitted for a, b in zip(rs, rs[1:]))


def test_coupled_time_steps(setup, ora):
    """Served steps coupled as the model's sea-surface step: each request's
    right-hand side is eq. (8)'s from that step's transports, its first guess
    2 D^{t-1} - D^{t-2} from the grid's previous solutions, and the heights
    follow eq. (1); checked against the oracle's passes on the host."""
    P, serve, probs = setup
    say("coupled time steps: 15 requests on 3 grids")
    srv = serve.Server(probs, drop_tol=0.1, device="cuda", chunk=8)
    reqs = serve.poisson_arrivals(rate=400.0, count=15, n_grids=len(probs), seed=11)
    stepper = serve.CoupledTimeStepper(probs, srv.solvers, torch.device("cuda"), seed=5,
                                       guess=(2.0, -1.0), dt=0.5)
    done = srv.run(reqs, make_rhs=stepper, on_done=stepper.done)
    assert len(done) == 15
    by_grid = {}
    for r in sorted(done, key=lambda r: r.step):
        by_grid.setdefault(r.grid, []).append(r)
    for g, rs in by_grid.items():
        p = probs[g]
        assert [r.step for r in rs] == list(range(len(rs)))
        eta = [np.zeros(p.n), np.zeros(p.n)]
        for r in rs:
            e2u, mu, e1v, mv = orca.orca_transports(p, r.step, seed=5)
            want_b = ora.ts_rhs(p.nx, p.ny, p.periodic, e2u, mu, e1v, mv)
            b = r.b.cpu().numpy()
            assert np.allclose(b, want_b, rtol=0, atol=1e-15 * np.abs(want_b).max())
            x = r.x.cpu().numpy()
            assert r.status == 0
            assert np.linalg.norm(b - ora.spmv(p, x)) <= 1e-10 * np.linalg.norm(b)
            if r.step >= 2:
                x1, x2 = rs[r.step - 1].x.cpu().numpy(), rs[r.step - 2].x.cpu().numpy()
                assert np.array_equal(r.x0.cpu().numpy(), ora.ts_guess(x1, x2, 2.0, -1.0))
            eta = [eta[1], ora.ts_eta(eta[0], x, 0.5)]
        got = stepper.eta[g][1].cpu().numpy()
        assert np.array_equal(got, eta[1])
        say("  grid", g, "steps", len(rs), "inner iterations", [r.inner for r in rs])


def test_solo_lane_for_large_grids(setup, ora):
    """Grids at or above solo_cells are served by a lane of their own (the
    single-grid mixed solve on a host thread) while the others share a batch:
    every result meets the FP64 target, equals the same solve run alone bit
    for bit, steps of one grid stay sequential, and the lane's work overlaps
    the batch's."""
    P, serve, probs = setup
    big = orca.orca_problem(182, 149, 200)
    grids = probs + [big]
    say("solo lane: 182x149 beside 3 batched grids")
    srv = serve.Server(grids, drop_tol=0.1, device="cuda", chunk=8, solo_cells=20_000)
    try:
        assert srv.solo == [False, False, False, True]
        reqs = serve.poisson_arrivals(rate=300.0, count=16, n_grids=len(grids), seed=13)
        stepper = serve.TimeStepper(grids, torch.device("cuda"), seed=6)
        done = srv.run(reqs, make_rhs=stepper, on_done=stepper.done)
        assert len(done) == 16 and srv.in_flight_bytes == 0 and not any(srv.busy)
        solo = [r for r in done if r.grid == 3]
        assert solo
        for r in done:
            p = grids[r.grid]
            b, x = r.b.cpu().numpy(), r.x.cpu().numpy()
            assert r.status == 0
            assert np.linalg.norm(b - ora.spmv(p, x)) / np.linalg.norm(b) <= 1e-10
            if r.grid == 3:
                alone = srv.solvers[3].solve_mixed(r.b, x0=r.x0, tol=srv.tol,
                                                   inner_tol=srv.inner_tol,
                                                   max_outer=srv.max_outer, refine=srv.refine)
                assert torch.equal(alone.x, r.x)
        rs = sorted(solo, key=lambda r: r.admitted)
        assert all(a.finished <= b.admitted for a, b in zip(rs, rs[1:]))
        others = [r for r in done if r.grid != 3]
        overlap = sum(any(o.admitted < s.finished and o.finished > s.admitted for o in others)
                      for s in solo)
        say("  solo steps", len(solo), "overlapping batched steps", overlap,
            "per class", serve.latency_stats(done, srv.klass)["per_class"])
        assert overlap > 0
    finally:
        srv.close()
