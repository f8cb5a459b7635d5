"""Host logic of the serving layer (no GPU): seeded arrival processes."""
import numpy as np
import pytest

from paper_1210_1878_amd import serve


def test_poisson_per_grid_counts_order_and_seed():
    rates, horizon = [50.0, 5.0, 0.0, 200.0], 20.0
    a = serve.poisson_arrivals_per_grid(rates, horizon, seed=11)
    b = serve.poisson_arrivals_per_grid(rates, horizon, seed=11)
    assert [(r.grid, r.arrival) for r in a] == [(r.grid, r.arrival) for r in b]
    t = [r.arrival for r in a]
    assert t == sorted(t) and all(0.0 <= x < horizon for x in t)
    assert [r.rid for r in a] == list(range(len(a)))
    for g, lam in enumerate(rates):
        k = sum(1 for r in a if r.grid == g)
        mean = lam * horizon
        assert abs(k - mean) <= 5 * np.sqrt(mean) + 1e-9     # Poisson count, 5 sigma
    # exponential gaps: the mean gap of the busiest grid is 1/rate
    t3 = np.array([r.arrival for r in a if r.grid == 3])
    assert abs(np.diff(t3).mean() * rates[3] - 1.0) < 0.1


def test_poisson_uniform_grids():
    a = serve.poisson_arrivals(rate=100.0, count=2000, n_grids=4, seed=3)
    t = np.array([r.arrival for r in a])
    assert np.all(np.diff(t) > 0)
    assert abs(t[-1] / 2000 * 100.0 - 1.0) < 0.1
    counts = np.bincount([r.grid for r in a], minlength=4)
    assert counts.min() > 400


def test_latency_stats_per_class():
    reqs = []
    for i in range(100):
        r = serve.Request(rid=i, grid=i % 3, arrival=0.01 * i)
        r.finished = r.arrival + (1.0 if r.grid == 2 else 0.01 * (1 + i % 7))
        r.status, r.true_relres = 0, 1e-11
        reqs.append(r)
    st = serve.latency_stats(reqs, klass=[0, 0, 1])
    assert st["requests"] == 100 and st["all_ok"]
    per = st["per_class"]
    assert per["0"]["requests"] + per["1"]["requests"] == 100
    assert abs(per["1"]["p50_ms"] - 1000.0) < 1e-6 and per["0"]["max_ms"] <= 70.0 + 1e-9
    # 67 and 33 samples per class: below the floor for a p99; 100 overall
    assert per["0"]["p99_ms"] is None and per["1"]["p99_ms"] is None
    assert st["p99_ms"] == pytest.approx(1000.0)


def _host_server(item_bytes, budget):
    """A Server with its host state only (no device): enough to run the
    admission loop on requests that are all rejected."""
    srv = object.__new__(serve.Server)
    srv.item_bytes = list(item_bytes)
    srv.budget = budget
    srv.klass = [0] * len(item_bytes)
    srv.busy = [False] * len(item_bytes)
    srv.batches = {}
    srv.in_flight_bytes = 0
    srv.max_slots = 4
    srv.solvers = [None] * len(item_bytes)
    return srv


def test_request_larger_than_budget_is_rejected_not_queued():
    """A request whose vectors alone exceed the budget can never be admitted:
    it is returned at arrival with status REJECTED (the loop must end)."""
    srv = _host_server([100, 5000], budget=1000)
    assert srv.can_ever_fit(0) and not srv.can_ever_fit(1)
    reqs = [serve.Request(rid=i, grid=1, arrival=0.001 * i) for i in range(5)]
    calls = []
    done = srv.run(reqs, make_rhs=lambda r: pytest.fail("must not admit"),
                   on_done=calls.append)
    assert len(done) == 5 and all(r.status == serve.REJECTED for r in done)
    assert calls == [] and srv.in_flight_bytes == 0
    st = serve.latency_stats(done)
    assert st == {"requests": 0, "rejected": 5}
    with pytest.raises(ValueError):
        srv.saturate(0.1, make_rhs=lambda r: None)
    srv.budget = None
    assert srv.can_ever_fit(1)


def test_latency_stats_counts_and_p99_floor():
    reqs = []
    for i in range(150):
        r = serve.Request(rid=i, grid=0 if i < 120 else 1, arrival=0.0)
        r.finished = 0.001 * (i + 1)
        r.status, r.true_relres = 0, 1e-11
        reqs.append(r)
    st = serve.latency_stats(reqs, klass=[0, 1], per_grid=True)
    assert st["p99_ms"] is not None and st["rejected"] == 0
    assert st["per_class"]["0"]["requests"] == 120 and st["per_class"]["0"]["p99_ms"] is not None
    assert st["per_class"]["1"]["requests"] == 30 and st["per_class"]["1"]["p99_ms"] is None
    assert st["per_grid"]["1"]["max_ms"] == pytest.approx(150.0)
