"""Continuous-batching server for the elliptic solve of successive time steps.

Each request is one time step of one grid: a right-hand side and a warm
start from the grid's previous solutions (the initial guess of Algorithm 1).
CoupledTimeStepper produces them as the model's sea-surface step does
(eq. (8) right-hand side from face transports, eq. (1) height update);
TimeStepper is a lighter stand-in (noise on the previous right-hand side).  Every grid's operator, D^-1 and Z stay
resident on the device (one PCGA_MIXED solver per grid).  Requests are
admitted as soon as their grid is idle (time steps of one grid are
sequential) and their vectors fit the device-memory budget.  Grids are split
into size classes, each with its own batch on its own HIP stream: a batch
advances all of its admitted requests together (one launch per kernel per
step), and the classes run concurrently, so that steps of a very large grid
do not hold back the many steps a small grid's solve needs.  Grids of at
least `solo_cells` cells are not batched: each has a lane of its own, a host
thread that runs the grid's steps through the single-grid mixed solve on the
grid's stream (its kernels stream the large grid's arrays better than the
batched kernels do), concurrently with the batches.  Latency is measured
from arrival to the moment the solution is back in the request's output
tensor.  The classes and lanes only overlap when their streams reach
different hardware queues: the runtime gives a process a fixed number of
them (GPU_MAX_HW_QUEUES, 4 by default, set before the runtime starts) and
binds each new stream to the queue with the fewest streams.  The server
makes the streams of its classes and lanes itself, one after the other
(HwStream), so that they land on distinct queues whatever streams the
process made before; torch's pooled streams, made in one burst when the
pool starts, share queues in an order that depends on the queue count.
"""
from __future__ import annotations

import collections
import dataclasses
import queue as _queue
import threading
import time

import numpy as np

from .api import Batch, HwStream, Solver, Stencil5, ainv_setup


REJECTED = -5   # the request's vectors alone exceed the memory budget (PCGA_ENOMEM)


@dataclasses.dataclass
class Request:
    rid: int
    grid: int
    arrival: float                 # seconds since the start of the run
    b: object = None               # device tensor [n]
    x0: object = None              # device tensor [n]
    admitted: float = -1.0
    finished: float = -1.0
    status: int = -99
    true_relres: float = float("nan")
    outer: int = 0
    inner: int = 0
    x: object = None

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


class _SoloLane:
    """One grid served outside the batches: a host thread that solves the
    grid's admitted steps one at a time with the single-grid mixed solve
    (the library releases the interpreter while it runs) and posts each
    finished request to the server's completion queue."""

    def __init__(self, solver, server, done_q):
        self.S = solver
        self.srv = server
        self.done_q = done_q
        self.inbox = _queue.Queue()
        self.thread = threading.Thread(target=self._loop, daemon=True)
        self.thread.start()

    def submit(self, req):
        self.inbox.put(req)

    def _loop(self):
        while True:
            req = self.inbox.get()
            if req is None:
                return
            srv = self.srv
            try:
                res = self.S.solve_mixed(req.b, x0=req.x0, tol=srv.tol, inner_tol=srv.inner_tol,
                                         max_outer=srv.max_outer, refine=srv.refine)
                q = {"status": res.status, "true_relres": [res.true_relres], "outer": res.outer,
                     "inner_total": res.inner_total}
                self.done_q.put((req, res.x.unsqueeze(0), q))
            except Exception as e:     # reported as a failed request, the lane goes on
                self.done_q.put((req, None, {"status": -4, "true_relres": [float("nan")],
                                             "outer": 0, "inner_total": 0, "error": repr(e)}))

    def close(self):
        self.inbox.put(None)
        self.thread.join(timeout=60)


class Server:
    """Holds resident grids and serves time-step solves by continuous batching."""

    def __init__(self, problems, drop_tol=0.05, device=None, hbm_budget=None, max_slots=64,
                 tol=1e-10, inner_tol=None, max_outer=None, chunk=16, class_cells=(2_000_000,),
                 class_grid=None, solo_cells=None, refine="keep"):
        import torch
        self.torch = torch
        self.device = torch.device("cuda" if device is None else device)
        # refinement of every solve: "keep" (inner direction kept across
        # corrections, runs of one decade) or "restart" (inner stop 1e-5)
        keep = refine == "keep"
        self.refine = refine
        self.tol = tol
        self.inner_tol = inner_tol if inner_tol is not None else (0.1 if keep else 1e-5)
        self.max_outer = max_outer if max_outer is not None else (200 if keep else 30)
        # size class of each grid: index of the first bound above its cell count;
        # grids of at least solo_cells cells form the last class, one lane each
        bounds = sorted(class_cells)
        self.klass = [sum(1 for c in bounds if p.nx * p.ny >= c) for p in problems]
        self.solo = [solo_cells is not None and p.nx * p.ny >= solo_cells for p in problems]
        solo_class = len(bounds) + 1
        self.klass = [solo_class if so else k for k, so in zip(self.klass, self.solo)]
        used = sorted({k for k, so in zip(self.klass, self.solo) if not so})
        # one stream per batch class and per lane, made together (distinct
        # hardware queues); the other grids' solvers take pooled streams
        self.hw_streams = {("batch", k): HwStream(self.device) for k in used}
        self.hw_streams.update({("solo", g): HwStream(self.device)
                                for g, so in enumerate(self.solo) if so})
        self.solvers = []
        self.resident_bytes = 0
        for g, p in enumerate(problems):
            A = Stencil5.from_problem(p)
            hs = self.hw_streams.get(("solo", g))
            S = Solver(A, ainv_setup(A, drop_tol), "mixed", device=self.device,
                       stream=None if hs is None else hs.torch)
            self.solvers.append(S)
            self.resident_bytes += S.footprint_bytes
        self.item_bytes = [Batch.item_bytes(S, 1) for S in self.solvers]
        self.budget = hbm_budget            # bytes for in-flight request vectors (None: no limit)
        self.max_slots = max_slots
        # class_grid: workgroups per launch of each class's batch (None: 2048),
        # so that a large grid's kernels can leave CUs to the other classes
        grids = class_grid or {}
        self.batches = {k: Batch(max_slots=max_slots, device=self.device, chunk=chunk,
                                 stream=self.hw_streams[("batch", k)].torch,
                                 grid=grids.get(k)) for k in used}
        self.in_flight_bytes = 0
        self.busy = [False] * len(self.solvers)
        self._solo_done = _queue.Queue()
        self.lanes = {g: _SoloLane(S, self, self._solo_done)
                      for g, (S, so) in enumerate(zip(self.solvers, self.solo)) if so}
        self._solo_flying = 0

    def close(self):
        """Stops the lanes, then releases the batches, the solvers and the
        streams (the server cannot serve afterwards)."""
        for lane in self.lanes.values():
            lane.close()
        self.lanes = {}
        for B in self.batches.values():
            B.close()
        for S in self.solvers:
            S.close()
        for hs in self.hw_streams.values():
            hs.close()
        self.hw_streams = {}

    def fits(self, grid):
        return self.budget is None or self.in_flight_bytes + self.item_bytes[grid] <= self.budget

    def can_ever_fit(self, grid):
        """Whether a request of this grid fits the budget with nothing else in
        flight; one that cannot is rejected at arrival instead of waiting
        forever."""
        return self.budget is None or self.item_bytes[grid] <= self.budget

    def _reject(self, req, now):
        req.admitted = now
        req.finished = now
        req.status = REJECTED

    def admit(self, req, now):
        k = self.klass[req.grid]
        if self.solo[req.grid]:
            self.in_flight_bytes += self.item_bytes[req.grid]
            self.busy[req.grid] = True
            req.admitted = now
            self._solo_flying += 1
            self.lanes[req.grid].submit(req)
            return ("solo", req.rid)
        slot = self.batches[k].add(self.solvers[req.grid], req.b.unsqueeze(0),
                                   X0=req.x0.unsqueeze(0), tol=self.tol,
                                   inner_tol=self.inner_tol, max_outer=self.max_outer, tag=req.rid,
                                   refine=self.refine)
        self.in_flight_bytes += self.item_bytes[req.grid]
        self.busy[req.grid] = True
        req.admitted = now
        return (k, slot)

    def _advance(self, slots, poll_chunks):
        """Launch every class batch that has work and no launch in flight, then
        collect one that finished.  Returns the finished (key, req, X, q)."""
        for k, B in self.batches.items():
            if k not in self._flying and any(key[0] == k for key in slots):
                B.launch(poll_chunks)
                self._flying.add(k)
        while True:
            out = []
            while True:
                try:
                    req, X, q = self._solo_done.get_nowait()
                except _queue.Empty:
                    break
                self._solo_flying -= 1
                out.append((("solo", req.rid), X, q))
            if out:
                return out
            for k in list(self._flying):
                ready, _ = self.batches[k].wait(block=False)
                if not ready:
                    continue
                self._flying.discard(k)
                out = []
                for key in [key for key in slots if key[0] == k]:
                    q = self.batches[k].query(key[1])
                    if q["done"]:
                        X, q = self.batches[k].remove(key[1])
                        out.append((key, X, q))
                return out
            time.sleep(20e-6)

    def _finish(self, req, X, q, now):
        req.finished = now
        req.status = q["status"]
        req.true_relres = q["true_relres"][0]
        req.outer, req.inner = q["outer"], q["inner_total"]
        req.x = X[0] if X is not None else None
        self.busy[req.grid] = False
        self.in_flight_bytes -= self.item_bytes[req.grid]

    def run(self, requests, make_rhs, on_done=None, clock=time.perf_counter, poll_chunks=1):
        """Serve `requests` (sorted by arrival).  make_rhs(req) fills req.b and
        req.x0 when the request is admitted (it may use the grid's previous
        solution); on_done(req) is called when a solution is back.
        Returns the finished requests; a request whose grid's vectors alone
        exceed the memory budget is returned at once with status REJECTED
        and no solution (on_done is not called for it)."""
        t0 = clock()
        pending = collections.deque(requests)
        queue = []
        slots = {}
        done = []
        self._flying = set()
        held = set()            # requests that waited for memory at least once
        while pending or queue or slots:
            now = clock() - t0
            while pending and pending[0].arrival <= now:
                req = pending.popleft()
                if self.can_ever_fit(req.grid):
                    queue.append(req)
                else:
                    self._reject(req, clock() - t0)
                    done.append(req)
            # admission: FIFO among requests whose grid is idle and that fit;
            # a class batch takes new items only between its launches
            rest = []
            for req in queue:
                k = self.klass[req.grid]
                free = (self.solo[req.grid] or
                        (k not in self._flying
                         and sum(1 for key in slots if key[0] == k) < self.batch_capacity()))
                if not self.busy[req.grid] and free and self.fits(req.grid):
                    make_rhs(req)
                    slots[self.admit(req, clock() - t0)] = req
                else:
                    if not self.busy[req.grid] and free:
                        held.add(req.rid)
                    rest.append(req)
            queue = rest
            if not slots:
                if pending:
                    wait = pending[0].arrival - (clock() - t0)
                    if wait > 0:
                        time.sleep(min(wait, 0.05))
                continue
            for key, X, q in self._advance(slots, poll_chunks):
                req = slots.pop(key)
                self._finish(req, X, q, clock() - t0)
                done.append(req)
                if on_done:
                    on_done(req)
        self._drain()
        self.held_for_memory = len(held)
        return done

    def _drain(self):
        for k in list(self._flying):
            self.batches[k].wait(block=True)
        self._flying = set()

    def batch_capacity(self):
        return self.max_slots

    def saturate(self, seconds, make_rhs, on_done=None, clock=time.perf_counter, poll_chunks=1):
        """Closed loop: every grid always has one time step in flight (the next
        is submitted as soon as the previous is back) until `seconds` have
        passed; then the steps in flight are drained.  Returns the finished
        requests and the elapsed time; completions per grid over the elapsed
        time are the grids' saturated throughputs."""
        t0 = clock()
        slots = {}
        done = []
        rid = [0]
        self._flying = set()
        too_big = [g for g in range(len(self.solvers)) if not self.can_ever_fit(g)]
        if too_big:
            raise ValueError(f"grids {too_big}: one request exceeds the memory budget")
        waiting = list(range(len(self.solvers)))   # grids whose next step is due

        def submit(g):
            now = clock() - t0
            req = Request(rid=rid[0], grid=g, arrival=now)
            rid[0] += 1
            make_rhs(req)
            slots[self.admit(req, clock() - t0)] = req

        while slots or waiting:
            for g in [g for g in waiting if self.solo[g] or self.klass[g] not in self._flying]:
                waiting.remove(g)
                submit(g)
            if not slots:
                continue
            for key, X, q in self._advance(slots, poll_chunks):
                req = slots.pop(key)
                self._finish(req, X, q, clock() - t0)
                done.append(req)
                if on_done:
                    on_done(req)
                if req.finished < seconds:
                    waiting.append(req.grid)
        self._drain()
        return done, clock() - t0


def poisson_arrivals(rate, count, n_grids, seed):
    """Seeded Poisson process: exponential gaps at `rate` per second, grids
    drawn uniformly."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, size=count))
    g = rng.integers(0, n_grids, size=count)
    return [Request(rid=i, grid=int(g[i]), arrival=float(t[i])) for i in range(count)]


def poisson_arrivals_per_grid(rates, horizon, seed):
    """Independent seeded Poisson processes, one per grid (rates[g] per
    second), over [0, horizon) seconds; merged in arrival order."""
    rng = np.random.default_rng(seed)
    ev = []
    for g, lam in enumerate(rates):
        t = 0.0
        while lam > 0:
            t += rng.exponential(1.0 / lam)
            if t >= horizon:
                break
            ev.append((t, g))
    ev.sort()
    return [Request(rid=i, grid=g, arrival=t) for i, (t, g) in enumerate(ev)]


class TimeStepper:
    """Per-grid right-hand sides of successive time steps and warm starts:
    b_t = b_{t-1} + 0.01 rms(b_{t-1}) xi, xi ~ N(0,1) on ocean cells (seeded),
    x0_t = x_{t-1} (zero for the first step)."""

    def __init__(self, problems, device, seed):
        import torch
        self.torch = torch
        self.device = device
        self.b = [torch.from_numpy(p.b.copy()).to(device) for p in problems]
        self.ocean = [torch.from_numpy(p.ocean.astype(np.float64)).to(device) for p in problems]
        self.x = [torch.zeros(p.n, dtype=torch.float64, device=device) for p in problems]
        self.gen = torch.Generator(device=device).manual_seed(seed)
        self.steps = [0] * len(problems)

    def __call__(self, req):
        g = req.grid
        if self.steps[g] > 0:
            b = self.b[g]
            xi = self.torch.randn(b.shape[0], generator=self.gen, dtype=self.torch.float64,
                                  device=self.device)
            rms = self.torch.sqrt((b * b).sum() / self.ocean[g].sum())
            self.b[g] = b + 0.01 * rms * xi * self.ocean[g]
        self.steps[g] += 1
        req.b = self.b[g].clone()
        req.x0 = self.x[g].clone()

    def done(self, req):
        self.x[req.grid] = req.x.clone()


class CoupledTimeStepper:
    """Successive time steps coupled as in the model's sea-surface step: the
    right-hand side of step t is eq. (8)'s, from that step's face transports
    (seeded, slowly varying; gen.orca.orca_transport_modes), the first guess is
    x0 = a D^{t-1} + c D^{t-2} from the grid's two previous solutions (the
    paper writes x0 = 2 D^{t-1}; with one previous solution x0 = D^{t-1}, with
    none x0 = 0), and each solution advances the sea-surface height by
    eq. (1), eta^{n+1} = eta^{n-1} - 2 dt D^n.  The right-hand side, the first
    guess and the height update run in the library's time-step passes on the
    grid's solver; the transports of a step are formed on the device from the
    modes (input synthesis)."""

    def __init__(self, problems, solvers, device, seed, guess=(2.0, -1.0), dt=0.5):
        import torch
        from gen import orca
        self.torch = torch
        self.device = device
        self.solvers = solvers
        self.guess = guess
        self.dt = dt
        dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(device)
        self.modes = []
        for p in problems:
            m = orca.orca_transport_modes(p, seed)
            self.modes.append({"w": list(m.w), "base_u": dev(m.base_u), "cu": [dev(a) for a in m.cu],
                               "su": [dev(a) for a in m.su], "cv": [dev(a) for a in m.cv],
                               "sv": [dev(a) for a in m.sv], "e2u": dev(m.e2u), "e1v": dev(m.e1v)})
        self.D = [[] for _ in problems]
        self.eta = [[torch.zeros(p.n, dtype=torch.float64, device=device) for _ in range(2)]
                    for p in problems]
        self.steps = [0] * len(problems)

    def transports(self, g, t):
        m = self.modes[g]
        mu = m["base_u"].clone()
        mv = self.torch.zeros_like(mu)
        for w, cu, su, cv, sv in zip(m["w"], m["cu"], m["su"], m["cv"], m["sv"]):
            c, s = np.cos(w * t), np.sin(w * t)
            mu += c * cu + s * su
            mv += c * cv + s * sv
        return mu, mv

    def __call__(self, req):
        g = req.grid
        S = self.solvers[g]
        req.step = self.steps[g]
        mu, mv = self.transports(g, self.steps[g])
        m = self.modes[g]
        req.b = S.ts_rhs(m["e2u"], mu, m["e1v"], mv)
        D = self.D[g]
        a, c = self.guess
        if not D:
            req.x0 = self.torch.zeros_like(req.b)
        elif len(D) == 1 or c == 0.0:
            req.x0 = S.ts_guess(D[-1], None, a if c == 0.0 else 1.0, 0.0)
        else:
            req.x0 = S.ts_guess(D[-1], D[-2], a, c)
        self.steps[g] += 1

    def done(self, req):
        g = req.grid
        x = req.x.clone()
        self.D[g] = (self.D[g] + [x])[-2:]
        e = self.eta[g]
        self.eta[g] = [e[1], self.solvers[g].ts_eta(e[0], x, self.dt)]


P99_MIN_SAMPLES = 100   # fewer samples than this: no p99 is quoted (None)


def _pct(lat_s, q):
    return float(np.percentile(lat_s, q) * 1e3)


def latency_stats(done, klass=None, per_grid=False):
    """Latency percentiles (arrival to solution) and throughput; with
    klass[grid] also per size class, with per_grid also per grid.  Every
    group reports its sample count; its p99 is None below P99_MIN_SAMPLES
    samples.  Rejected requests are counted, not timed."""
    rejected = sum(1 for r in done if r.status == REJECTED)
    done = [r for r in done if r.status != REJECTED]
    if not done:
        return {"requests": 0, "rejected": rejected}
    lat = np.array([r.latency for r in done])
    span = max(r.finished for r in done) - min(r.arrival for r in done)
    out = {"requests": len(done), "rejected": rejected, "p50_ms": _pct(lat, 50),
           "p99_ms": _pct(lat, 99) if len(lat) >= P99_MIN_SAMPLES else None,
           "mean_ms": float(lat.mean() * 1e3),
           "solves_per_s": len(done) / span if span > 0 else float("nan"),
           "worst_true_relres": float(max(r.true_relres for r in done)),
           "all_ok": all(r.status == 0 for r in done)}
    def group(sel):
        lk = np.array([r.latency for r in done if sel(r)])
        if not len(lk):
            return None
        return {"requests": int(len(lk)), "p50_ms": _pct(lk, 50),
                "p99_ms": _pct(lk, 99) if len(lk) >= P99_MIN_SAMPLES else None,
                "max_ms": float(lk.max() * 1e3)}

    if klass is not None:
        per = {}
        for k in sorted(set(klass)):
            g = group(lambda r: klass[r.grid] == k)
            if g:
                per[str(k)] = g
        out["per_class"] = per
    if per_grid:
        out["per_grid"] = {str(gi): group(lambda r: r.grid == gi)
                           for gi in sorted({r.grid for r in done})}
    return out
