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
    assert abs(per["1"]["p50_ms"] - 1000.0) < 1e-6 and per["0"]["p99_ms"] <= 70.0 + 1e-9
    assert st["p99_ms"] == pytest.approx(1000.0)
