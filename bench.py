#!/usr/bin/env python3
"""Benchmark: PCG-AINV iterations/s on the 1442x1021 ORCA025-shaped grid.

One step = one full FP64 PCG-AINV solve (Algorithm 1, P = Z D^-1 Z^T, drop
tolerance 0.05) of the synthetic 1442x1021 problem from x0 = 0 to relative
residual 1e-10, inputs resident in HBM.  `value` = iterations per second over
the K timed steps.  The same JSON line carries the mixed-precision solve (FP32
inner PCG + FP64 refinement) on the same GPU, the diagonal (Jacobi)
preconditioner baseline, the paper's banded factor of T (q = 4), the fixed-fill
AINV (the second Bridson class of Sec. 5), a general sparse (CSR) operator, the
roofline of the dominant kernel (HIP-event timing on the solver stream) and of
the whole iteration, the batched and served workloads with their modelled
bandwidth, and the FP64 oracle timed on the host.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)
# The runtime maps a process's streams round-robin onto its hardware queues
# (4 by default).  The served workload runs a batch per size class and a
# lane per large grid, each on its own stream, in a process that has created
# many solver streams before: with 4 queues some of them share a queue and
# run one after the other (closed-loop capacity 12.2 against 27.5 solves/s
# with 16).  Set before the runtime starts.
os.environ.setdefault("GPU_MAX_HW_QUEUES", "16")

NX, NY, TAU, TOL = 1442, 1021, 0.05, 1e-10
# fixed-fill AINV settings reported beside the threshold factor: (drop_tol, count)
FIXED_FILL = ((0.01, 8),)
SAMPLE_TOL = 1e-14      # stopping tolerance of the oracle's timed samples
KEEP_SEGMENT = 0.1      # residual reduction of one inner run when the direction is kept
PLACEMENTS = 1          # workspace bases the FP64 solver tries (1: the aligned base alone)
PEAK_HBM_GBS = 8000.0
METRIC = "PCG iter/s + HBM GB/s @1442x1021 FP64 vs mixed; served solves/s, p99 lat"


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


FMT_NT_X, FMT_X_DEF = 8, 16   # Z^T format bits: x streamed; x += alpha d in the stencil


def x_in_stencil(S):
    return bool(S.formats[0] & FMT_X_DEF)


def kernel_names(word, formats):
    """Iteration kernels as rocprofv3 names them (template arguments: value
    type, fused/dot flags, storage/read format of Z^T and Z; the stencil's
    coefficient type and x-update mode when the solver reports the update
    moved into the stencil: 1, 2 with x streamed)."""
    t = "double" if word == 8 else "float"
    f0 = formats[0]
    if f0 & FMT_X_DEF:
        xd = 2 if f0 & FMT_NT_X else 1
        return {"stencil": f"k_stencil<{t}, false, double, {xd}>",
                "axpy_zt": f"k_zt<{t}, true, {f0 & ~FMT_NT_X}>",
                "z_dot": f"k_z<{t}, true, false, {formats[1]}>"}
    return {"stencil": f"k_stencil<{t}, false, double, 0>", "axpy_zt": f"k_zt<{t}, true, {f0}>",
            "z_dot": f"k_z<{t}, true, false, {formats[1]}>"}


def kernel_bytes(n, nnz_off, word, index_bytes=4, x_in_stencil=False):
    """Algorithmic bytes per launch of the three iteration kernels (each array
    once; a Z entry = its value + its index: a 4-byte column or a 2-byte
    distance).  word = 8 (FP64) or 4 (FP32).  x_in_stencil: x += alpha d
    done by the stencil (x read and written there; d and x not touched by
    the Z^T kernel)."""
    e = word + index_bytes
    if x_in_stencil:
        return {
            "stencil": 6 * word * n + 24 * n,      # s, d_old, x in; d, q, x out; FP64 diag, ae, an
            "axpy_zt": 5 * word * n + e * nnz_off,  # r, q, D^-1 in; r', t out; Z^T
            "z_dot": 3 * word * n + e * nnz_off,    # t, r' in; s out; Z
        }
    return {
        "stencil": 4 * word * n + 24 * n,      # s, d_old in; d, q out; FP64 diag, ae, an in
        "axpy_zt": 8 * word * n + e * nnz_off,  # r, q, d, x, D^-1 in; r', x, t out; Z^T
        "z_dot": 3 * word * n + e * nnz_off,    # t, r' in; s out; Z
    }


def survey_bytes(n, nnz_off, x_in_stencil=False):
    """Compulsory bytes of one FP64 iteration by method step (FP64 values,
    int32 column per nonzero of Z, each array counted once per step):
    direction update + five-point product + (d,q) 56 n; alpha, the two axpys
    and ||r||^2 48 n (r' = r - alpha q 24 n, x' = x + alpha d 24 n);
    t = D^-1 Z^T r 24 n + 12 nnz; s = Z t and (s,r) 24 n + 12 nnz.  The Z^T
    kernel fuses the second and third steps; with x_in_stencil the x axpy
    is done by the stencil instead."""
    xa = 24 * n if x_in_stencil else 0
    return {"stencil": 56 * n + xa, "axpy_zt": 48 * n - xa + 24 * n + 12 * nnz_off,
            "z_dot": 24 * n + 12 * nnz_off, "iteration": 152 * n + 24 * nnz_off}


def batch_step_bytes(n, nnz_stored, nrhs, index_bytes):
    """Compulsory bytes of one inner step of a batch slot (FP32 vectors
    interleaved over nrhs right-hand sides, FP64 operator, FP32 Z values):
    stencil 16 R n + 24 n; Z^T kernel 28 R n + 4 n + (4 + b) E; Z kernel
    12 R n + (4 + b) E."""
    return 56 * nrhs * n + 28 * n + 2 * (4 + index_bytes) * nnz_stored


COUNTER_FILE = os.path.join(ROOT, "profiles", "pcg_iteration_kernels_1442x1021_hbm_traffic.json")
TRACE_FILE = os.path.join(ROOT, "profiles", "pcg_iteration_kernels_1442x1021_trace.json")
KERNEL_SOURCES = ["paper_1210_1878_amd/csrc/kernels.h", "paper_1210_1878_amd/csrc/pcga_dev.h",
                  "paper_1210_1878_amd/csrc/solver.hip", "paper_1210_1878_amd/csrc/timestep.hip"]
# Time-step passes around the solve: algorithmic bytes per cell (each array once)
TS_KERNEL_BYTES = {"k_ts_rhs": 40,          # e2u, Mu, e1v, Mv in; b out
                   "k_ts_guess<true>": 24,  # D^{t-1}, D^{t-2} in; x0 out
                   "k_ts_eta": 24}          # eta^{n-1}, D^n in; eta^{n+1} out


def kernel_source_hash():
    """SHA-256 over the code of the sources that define the iteration kernels
    and their launch: comments and whitespace are removed first, so that an
    edit of a comment does not void counters taken on the same code."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), encoding="utf-8") as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)   # block comments
        text = re.sub(r"//[^\n]*", " ", text)                 # line comments
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE, each scaled by its reading on a plain
    device copy), or None when there is none or the kernel sources changed
    since the counters were taken."""
    try:
        with open(COUNTER_FILE) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None, "no counter summary"
    if rec.get("source_sha256") != kernel_source_hash():
        return None, "kernel sources changed since the counters were taken"
    k = rec.get("kernels", {}).get(kernel)
    if k is None:
        return None, "kernel not in the counter summary"
    return k["hbm_bytes_per_launch"], rec.get("profile", "")


def traced_us(kernel):
    """Average duration in us of `kernel` in the committed rocprofv3 kernel
    trace of `bench.py --kernels-only`, or None when the kernel sources
    changed since the trace was taken."""
    try:
        with open(TRACE_FILE) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("source_sha256") != kernel_source_hash():
        return None
    k = rec.get("kernels", {}).get(kernel)
    return None if k is None else k["avg_us"]


def cpu_baseline(p, seconds=15.0):
    """The FP64 oracle (single thread) on a bounded sample of the workload."""
    import oracle
    t0 = time.perf_counter()
    F = oracle.ainv_setup(p, TAU)
    setup_s = time.perf_counter() - t0
    # calibrate on a few iterations, then run a sample of ~`seconds`
    t0 = time.perf_counter()
    oracle.pcg(p, F, tol=SAMPLE_TOL, maxit=5)
    per_it = (time.perf_counter() - t0) / 5
    m = max(10, int(seconds / per_it))
    t0 = time.perf_counter()
    # a tolerance far below the solve's, not 0: a fast host could otherwise run
    # past convergence into a breakdown (rho or (d, q) reaching 0)
    r = oracle.pcg(p, F, tol=SAMPLE_TOL, maxit=m)
    dt = time.perf_counter() - t0
    return {"value": r.iters / dt, "unit": "iter/s", "cores": 1, "kind": "oracle",
            "sample": f"{r.iters} FP64 PCG-AINV iterations of the oracle on the 1442x1021 "
                      f"problem from x0=0 (setup {setup_s:.1f}s excluded), one thread",
            "setup_s": round(setup_s, 2), "host_cpu": host_cpu_model(),
            "host_threads": os.cpu_count(),
            "jacobi": cpu_jacobi(p, max(2.0, seconds / 5)),
            "ensemble": cpu_ensemble(max(2.0, seconds / 3))}


def cpu_jacobi(p, seconds):
    """The oracle's Jacobi PCG (drop tolerance +inf: Z = I, D = diag(A)) in
    the same harness: iterations per second on the same problem."""
    import oracle
    F = oracle.ainv_setup(p, float("inf"))
    t0 = time.perf_counter()
    oracle.pcg(p, F, tol=SAMPLE_TOL, maxit=5)
    m = max(10, int(seconds / ((time.perf_counter() - t0) / 5)))
    t0 = time.perf_counter()
    r = oracle.pcg(p, F, tol=SAMPLE_TOL, maxit=m)
    return {"value": round(r.iters / (time.perf_counter() - t0), 2), "unit": "iter/s",
            "sample": f"{r.iters} iterations"}


def cpu_ensemble(seconds, members=64, nrhs=4):
    """The oracle on the batched workload: whole FP64 solves to 1e-10 of the
    ensemble's grids and right-hand sides, in order, until about `seconds`
    have passed (setups excluded).  Reported per core, and as the aggregate of
    one independent solve per host thread (the ensemble's solves share
    nothing)."""
    import oracle
    from gen import orca
    ens = orca.ensemble_problems(count=members, nrhs=nrhs)
    done, busy = 0, 0.0
    for q in ens:
        F = oracle.ainv_setup(q, 0.1)
        for r in range(nrhs):
            t0 = time.perf_counter()
            oracle.pcg(q, F, b=q.B[r], tol=TOL)
            busy += time.perf_counter() - t0
            done += 1
        if busy >= seconds:
            break
    per_core = done / busy
    threads = os.cpu_count() or 1
    return {"solves_per_s_per_core": round(per_core, 2),
            "solves_per_s_all_threads": round(per_core * threads, 1),
            "sample": f"{done} of the {members * nrhs} ensemble solves (FP64, 1e-10), one thread; "
                      f"the aggregate assumes one independent solve per host thread"}


def host_cpu_model():
    """The host CPU's model name (Linux /proc/cpuinfo), or None."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def bench_batch(P, torch, dev, log, members=64, nrhs=4):
    """64 uneven ORCA-shaped grids x 4 right-hand sides, mixed precision to
    1e-10, advanced together by the batched kernels (one launch per kernel
    per iteration for the whole ensemble)."""
    from gen import orca
    from paper_1210_1878_amd import autotune
    t0 = time.perf_counter()
    ens = orca.ensemble_problems(count=members, nrhs=nrhs)
    As = [P.Stencil5.from_problem(p) for p in ens]
    Fs = [P.ainv_setup(A, 0.1) for A in As]
    Bs = [torch.from_numpy(p.B).to(dev) for p in ens]
    cells = sum(p.n for p in ens)
    log(f"ensemble: {members} grids, {cells} cells, setup {time.perf_counter() - t0:.1f}s")
    # slice width and chunk of the ensemble picked by timing whole batched solves
    t0 = time.perf_counter()
    tuned = autotune.tune_batch(
        lambda w: [(P.Solver(A, F, "mixed", device=dev, slice_width=w), B) for A, F, B in zip(As, Fs, Bs)],
        widths=(8, 16, 32), chunks=(8, 16, 32), tol=TOL, refine="keep")
    log(f"ensemble autotune ({time.perf_counter() - t0:.1f}s): slice width {tuned['slice_width']}, "
        f"chunk {tuned['chunk']}; " + ", ".join(f"w{w}/c{c}: {ms:.0f} ms" for w, c, ms in tuned["table"]))
    solvers = [P.Solver(A, F, "mixed", device=dev, slice_width=tuned["slice_width"]) for A, F in zip(As, Fs)]

    slot_of = {}

    def run_batch(refine):
        Bt = P.Batch(max_slots=members, device=dev, chunk=tuned["chunk"])
        for i, (S, B) in enumerate(zip(solvers, Bs)):
            slot_of[Bt.add(S, B, tol=TOL, refine=refine)] = i
        return Bt.solve()

    # restarted refinement (inner stop 1e-5 per correction), then the inner
    # direction kept across corrections (inner runs of one decade)
    run_batch("restart")                         # warm-up (graph capture)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res_r = run_batch("restart")
    torch.cuda.synchronize()
    dt_r = time.perf_counter() - t0
    inner_r = sum(q["inner_total"] for (_, q) in res_r.values())
    ok_r = all(q["status"] == 0 for (_, q) in res_r.values())
    worst_r = max(max(q["true_relres"]) for (_, q) in res_r.values())
    run_batch("keep")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = run_batch("keep")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    worst = max(max(q["true_relres"]) for (_, q) in res.values())
    ok = all(q["status"] == 0 for (_, q) in res.values())
    inner = sum(q["inner_total"] for (_, q) in res.values())
    # modelled bytes of all slot steps (inner steps; the few refinement steps
    # are left out, so the figure is a lower bound)
    moved = sum(q["inner_total"] * batch_step_bytes(solvers[slot_of[s]].n, solvers[slot_of[s]].nnz_off,
                                                    nrhs, solvers[slot_of[s]].index_bytes)
                for s, (_, q) in res.items())
    # the same solves one at a time through the single-grid mixed solver
    t0 = time.perf_counter()
    for S, B in zip(solvers, Bs):
        for r in range(nrhs):
            S.solve_mixed(B[r].contiguous(), tol=TOL, refine="keep")
    torch.cuda.synchronize()
    dts = time.perf_counter() - t0
    log(f"batched: {members * nrhs} solves in {dt * 1e3:.1f} ms ({members * nrhs / dt:.1f} solves/s), "
        f"worst true relres {worst:.2e}, all ok {ok}; restarted refinement {dt_r * 1e3:.1f} ms; "
        f"one at a time {dts * 1e3:.1f} ms")
    return {"workload": f"{members} uneven ORCA-shaped grids (182..362 x 149..292, own depth and "
                        f"land), {nrhs} RHS each, mixed precision to 1e-10, inner direction kept "
                        f"across corrections",
            "solves": members * nrhs, "cells": cells, "ms": round(dt * 1e3, 2),
            "solves_per_s": round(members * nrhs / dt, 1), "all_converged": ok,
            "worst_true_relres": worst, "inner_steps_per_slot": round(inner / members, 1),
            "restarted_refinement": {"ms": round(dt_r * 1e3, 2),
                                     "solves_per_s": round(members * nrhs / dt_r, 1),
                                     "inner_steps_per_slot": round(inner_r / members, 1),
                                     "all_converged": ok_r, "worst_true_relres": worst_r},
            "sequential_ms": round(dts * 1e3, 2),
            "speedup_vs_sequential": round(dts / dt, 2),
            "model_bytes": moved,
            "roofline": {"bound": "hbm", "achieved": round(moved / dt / 1e9, 1), "peak": PEAK_HBM_GBS,
                         "unit": "GB/s", "frac": round(moved / dt / 1e9 / PEAK_HBM_GBS, 4),
                         "model": "per slot inner step 56 R n + 28 n + 2 (4 + b) nnz_off bytes "
                                  "(R = 4 right-hand sides), summed over the slots' inner steps"},
            "autotuned": {"slice_width": tuned["slice_width"], "chunk": tuned["chunk"],
                          "table_ms": [[w, c, round(ms, 1)] for w, c, ms in tuned["table"]]}}


CSR_POINTS = 1_500_000


def bench_csr(P, torch, dev, log):
    """A general sparse SPD matrix that is not a grid (seeded unstructured
    point cloud, about 1.5 M rows, reverse Cuthill-McKee order), FP64
    PCG-AINV to 1e-10 through the CSR path."""
    from gen.unstructured import unstructured_problem
    t0 = time.perf_counter()
    q = unstructured_problem(CSR_POINTS, 1878 + 7)
    A = P.CsrMatrix.from_problem(q)
    G = P.ainv_setup(A, TAU)
    S = P.Solver(A, G, "fp64", device=dev)
    bq = torch.from_numpy(q.b).to(dev)
    log(f"csr: {q.n} rows, {q.nnz} entries, nnz_off(Z) {G.nnz_off}, setup {time.perf_counter() - t0:.1f}s")
    S.solve(bq, tol=TOL)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = S.solve(bq, tol=TOL)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ms = S.profile_iteration(bq, reps=50, mode=1)
    bpi = S.bytes_per_iter
    S.close()
    log(f"csr: {r.iters} iterations, {el * 1e3:.1f} ms, {r.iters / el:.0f} it/s, iteration "
        f"{ms[3] * 1e3:.1f} us ({bpi / (ms[3] * 1e-3) / 1e9:.0f} GB/s modelled), true relres "
        f"{r.true_relres:.2e}")
    return {"workload": f"unstructured point-cloud SPD matrix (k-nearest-neighbour couplings, "
                        f"RCM order), {q.n} rows, {q.nnz} entries, AINV drop tol {TAU}, FP64 to {TOL}",
            "n": q.n, "nnz": q.nnz, "nnz_off_z": G.nnz_off, "iters": r.iters,
            "ms_per_solve": round(el * 1e3, 2), "it_s": round(r.iters / el, 1),
            "true_relres": r.true_relres, "iteration_us": round(ms[3] * 1e3, 2),
            "kernel_us": [round(x * 1e3, 2) for x in ms[:3]],
            "model_bytes_per_iter": bpi,
            "model_gbs": round(bpi / (ms[3] * 1e-3) / 1e9, 1)}


SERVE_CLASS_CELLS = (2_000_000,)
SERVE_SOLO_CELLS = 1_000_000   # grids served by a lane of their own (single-grid mixed solve)
SERVE_BUDGET_FRAC = 0.6        # memory budget: the largest grid's request vectors plus this
                               # share of all other grids' (every grid fits alone, not all at once)


def serve_budget(item_bytes, frac=None):
    frac = SERVE_BUDGET_FRAC if frac is None else frac
    big = max(item_bytes)
    return int(big + frac * (sum(item_bytes) - big))
SERVE_GUESS = (2.0, -1.0)      # x0 = 2 D^{t-1} - D^{t-2}


def served_bytes(done, solvers):
    """Modelled bytes of the served requests' inner steps (one right-hand
    side; see batch_step_bytes)."""
    return sum(r.inner * batch_step_bytes(solvers[r.grid].n, solvers[r.grid].nnz_off, 1,
                                          solvers[r.grid].index_bytes)
               for r in done if r.status == 0)


def fp64_sequential(P, torch, dev, probs, seconds, log):
    """The same kind of requests served without batching and in FP64: every
    grid's next warm-started time step (1% noise on the right-hand side, x0 =
    the previous solution) solved in turn by a single-grid FP64 solver, until
    `seconds` have passed (at least one round).  Solves per second."""
    from paper_1210_1878_amd import serve
    solvers = [P.Solver(P.Stencil5.from_problem(p), P.ainv_setup(P.Stencil5.from_problem(p), 0.05),
                        "fp64", device=dev) for p in probs]
    stepper = serve.TimeStepper(probs, dev, seed=CONFIG_SERVE_SEED + 9)
    done, rid, cells = 0, 0, 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    while True:
        for g, S in enumerate(solvers):
            req = serve.Request(rid=rid, grid=g, arrival=0.0)
            rid += 1
            stepper(req)
            res = S.solve(req.b, req.x0, tol=TOL)
            req.x = res.x
            stepper.done(req)
            done += 1
            cells += probs[g].n
        if time.perf_counter() - t0 >= seconds:
            break
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    for S in solvers:
        S.close()
    log(f"fp64, one solve at a time: {done} solves in {el:.1f}s ({done / el:.2f} solves/s)")
    return {"solves": done, "seconds": round(el, 2), "solves_per_s": round(done / el, 2),
            "cells_per_s": round(cells / el, 1)}


def bench_serve(P, torch, dev, log, loads=(0.5, 0.8), saturate_s=6.0, horizon_s=15.0,
                class_cells=SERVE_CLASS_CELLS, coupled=False, compare_fp64=False,
                solo_cells=SERVE_SOLO_CELLS, budget_frac=None):
    """Time-step solves on a catalogue of resident grids from 182x149 to
    4322x3059 (mixed precision to 1e-10, warm starts, continuous batching).
    Capacity first: a closed loop keeps every grid busy and gives each grid's
    saturated throughput c_g.  Then, per load factor L, independent Poisson
    arrivals per grid at rate L * c_g over a fixed horizon; latency is arrival
    to solution."""
    from gen import orca
    from paper_1210_1878_amd import serve
    shapes = [(182, 149), (182, 149), (362, 292), (362, 292), (721, 510), (721, 510),
              (1442, 1021), (4322, 3059)]
    t0 = time.perf_counter()
    probs = [orca.orca_problem(nx, ny, orca.CONFIG_SEED_BASE + 40 + i) for i, (nx, ny) in enumerate(shapes)]
    srv = serve.Server(probs, drop_tol=0.05, device=dev, chunk=16, class_cells=class_cells,
                       solo_cells=solo_cells)
    srv.budget = serve_budget(srv.item_bytes, budget_frac)
    log(f"serving: {len(probs)} resident grids ({srv.resident_bytes / 2**30:.2f} GiB), "
        f"request-memory budget {srv.budget / 2**20:.0f} MiB, setup {time.perf_counter() - t0:.1f}s")
    if coupled:
        stepper = serve.CoupledTimeStepper(probs, srv.solvers, dev, seed=CONFIG_SERVE_SEED,
                                           guess=SERVE_GUESS)
    else:
        stepper = serve.TimeStepper(probs, dev, seed=CONFIG_SERVE_SEED)
    # warm-up: one step per grid (graph capture, first touch)
    warm = [serve.Request(rid=-1 - g, grid=g, arrival=0.0) for g in range(len(probs))]
    srv.run(warm, make_rhs=stepper, on_done=stepper.done)
    srv.budget = None        # the closed loop keeps every grid busy
    done, el = srv.saturate(saturate_s, make_rhs=stepper, on_done=stepper.done)
    srv.budget = serve_budget(srv.item_bytes, budget_frac)
    cap = [sum(1 for r in done if r.grid == g) / el for g in range(len(probs))]
    cap_bytes = served_bytes(done, srv.solvers)
    log(f"capacity (closed loop, {el:.1f}s): {sum(cap):.1f} solves/s; per grid "
        + ", ".join(f"{a}x{b}: {c:.2f}" for (a, b), c in zip(shapes, cap)))
    steps = ("coupled time steps (right-hand side of eq. (8) from seeded, slowly varying face "
             "transports; first guess x0 = 2 D^{t-1} - D^{t-2}; eq. (1) height update)" if coupled else
             "warm-started time steps (b_t = b_{t-1} + 1% seeded noise on ocean cells, x0 = x_{t-1})")
    out = {"workload": steps + " on 8 resident ORCA-shaped grids 182x149 .. 4322x3059, mixed "
                       "precision to 1e-10, continuous batching; per-grid Poisson arrivals at a "
                       "load factor of each grid's closed-loop throughput",
           "grids": [f"{a}x{b}" for a, b in shapes],
           "size_classes": "grids split at " + ", ".join(f"{c:,} cells" for c in sorted(class_cells))
                           + "; one batch per class, each on its own stream, running concurrently; "
                           f"grids of at least {solo_cells:,} cells are served by a lane of "
                           "their own (single-grid mixed solve on a host thread)",
           "grid_class": srv.klass,
           "solo_grids": [f"{a}x{b}" for (a, b), so in zip(shapes, srv.solo) if so],
           "hbm_budget_bytes": srv.budget,
           "capacity_solves_per_s": round(sum(cap), 2),
           "capacity_per_grid": [round(c, 3) for c in cap],
           # solves weighted by grid size (a 4322x3059 solve is 488 of 182x149)
           "capacity_cells_per_s": round(sum(c * p.n for c, p in zip(cap, probs)), 1),
           "refine": srv.refine,
           "capacity_worst_true_relres": float(max(r.true_relres for r in done)),
           "capacity_roofline": {"bound": "hbm", "achieved": round(cap_bytes / el / 1e9, 1),
                                 "peak": PEAK_HBM_GBS, "unit": "GB/s",
                                 "frac": round(cap_bytes / el / 1e9 / PEAK_HBM_GBS, 4),
                                 "model": "inner steps of the served solves x (56 n + 28 n + 2 (4 + b) "
                                          "nnz_off) bytes, over the closed-loop time"},
           "loads": {}}
    for i, L in enumerate(loads):
        reqs = serve.poisson_arrivals_per_grid([L * c for c in cap], horizon_s,
                                               seed=CONFIG_SERVE_SEED + 1 + i)
        # a progress line about every 30 s of a long horizon
        tick = {"t": time.perf_counter(), "n": 0}

        def on_done(req, tick=tick, total=len(reqs), L=L):
            stepper.done(req)
            tick["n"] += 1
            if time.perf_counter() - tick["t"] > 30.0:
                tick["t"] = time.perf_counter()
                log(f"load {L:.2f}: {tick['n']} of {total} requests done")
        res = srv.run(reqs, make_rhs=stepper, on_done=on_done)
        st = serve.latency_stats(res, srv.klass, per_grid=True)
        st["held_for_memory"] = srv.held_for_memory
        span = max(r.finished for r in res) - min(r.arrival for r in res)
        st["model_gbs"] = round(served_bytes(res, srv.solvers) / span / 1e9, 1)
        f99 = lambda v: "n/a" if v is None else f"{v:.0f}"
        log(f"load {L:.2f}: {st['requests']} requests, p50 {st['p50_ms']:.1f} ms, "
            f"p99 {f99(st['p99_ms'])} ms, {st['solves_per_s']:.2f} solves/s, "
            f"worst true relres {st['worst_true_relres']:.2e}; per size class "
            + ", ".join(f"{k}: {v['requests']} req p50 {v['p50_ms']:.0f} p99 {f99(v['p99_ms'])} ms"
                        for k, v in st["per_class"].items()))
        out["loads"][str(L)] = st
    if compare_fp64:
        out["fp64_one_at_a_time"] = fp64_sequential(P, torch, dev, probs, saturate_s, log)
        out["fp64_one_at_a_time"]["served_capacity_ratio"] = round(
            sum(cap) / out["fp64_one_at_a_time"]["solves_per_s"], 2)
        out["fp64_one_at_a_time"]["served_cells_ratio"] = round(
            out["capacity_cells_per_s"] / out["fp64_one_at_a_time"]["cells_per_s"], 2)
    srv.close()
    return out


CONFIG_SERVE_SEED = 1878 + 4
CONFIG_TS_SEED = 1878 + 5


def bench_timestep(P, torch, S, p, log, steps=10, dt_step=0.5):
    """Coupled time steps around the FP64 solve on the benchmark grid: per step
    the right-hand side of eq. (8) from that step's face transports (seeded,
    slowly varying), the first guess of Algorithm 1 from earlier solutions,
    the solve to 1e-10 and the sea-surface update of eq. (1).  Run once per
    reading of the first guess (the paper writes x0 = 2 D^{t-1}); iterations
    and time per step are averaged over the steps after the first two."""
    import numpy as np
    from gen import orca
    dev = torch.device("cuda:0")
    faces = [[torch.from_numpy(f).to(dev) for f in orca.orca_transports(p, t, CONFIG_TS_SEED)]
             for t in range(steps)]
    readings = {"zero": None, "previous": (1.0, 0.0), "printed_2D": (2.0, 0.0),
                "extrapolated": (2.0, -1.0)}
    res = {}
    for name, g in readings.items():
        zero = torch.zeros(p.n, dtype=torch.float64, device=dev)
        eta = [zero, zero.clone()]
        D, iters, times = [], [], []
        for t in range(steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            b = S.ts_rhs(*faces[t])
            if g is None or not D:
                x0 = None
            elif g[1] == 0.0:
                x0 = S.ts_guess(D[-1], None, g[0], 0.0)
            elif len(D) == 1:
                x0 = S.ts_guess(D[-1], None, 1.0, 0.0)
            else:
                x0 = S.ts_guess(D[-1], D[-2], g[0], g[1])
            r = S.solve(b, x0, tol=TOL)
            eta = [eta[1], S.ts_eta(eta[0], r.x, dt_step)]
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
            iters.append(r.iters)
            D = (D + [r.x])[-2:]
        res[name] = {"iters_per_step": iters, "mean_iters": round(float(np.mean(iters[2:])), 1),
                     "ms_per_step": round(float(np.mean(times[2:])) * 1e3, 2)}
    log(f"time steps ({steps}, 1442x1021, FP64): "
        + ", ".join(f"x0 {k}: {v['mean_iters']} it, {v['ms_per_step']} ms/step" for k, v in res.items()))
    return {"workload": f"{steps} coupled time steps on the 1442x1021 grid: b from seeded, slowly "
                        "varying face transports (eq. (8)), FP64 solve to 1e-10 from the first "
                        "guess of each reading, eta update (eq. (1)); means over steps 3..",
            "readings": res}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--chunk", type=int, default=32)
    ap.add_argument("--max-blocks", type=int, default=0,
                    help="workgroups per kernel; 0 = the solver's default (FP64 1280, mixed 1536)")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched ensemble")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving run")
    ap.add_argument("--no-timestep", action="store_true", help="skip the coupled time steps")
    ap.add_argument("--no-tune", action="store_true", help="skip the autotuner report")
    ap.add_argument("--no-csr", action="store_true", help="skip the general sparse operator")
    ap.add_argument("--serve-horizon", type=float, default=15.0,
                    help="seconds of Poisson arrivals per load factor in the serving runs")
    ap.add_argument("--serve-solo-cells", type=int, default=SERVE_SOLO_CELLS,
                    help="grids of at least this many cells get a serving lane of their own")
    ap.add_argument("--serve-budget-frac", type=float, default=SERVE_BUDGET_FRAC,
                    help="request-memory budget: the largest grid's vectors plus this share of "
                         "the other grids' (1: never binding)")
    ap.add_argument("--batch-only", action="store_true",
                    help="only the batched ensemble (for profiling its kernels)")
    ap.add_argument("--serve-only", action="store_true",
                    help="run only the two serving workloads (a long horizon gives the largest "
                         "grids enough requests) and print their results as one JSON line")
    ap.add_argument("--kernels-only", action="store_true",
                    help="profiling driver: a 256 MiB device copy (counter calibration), then the "
                         "three FP64 and FP32 iteration kernels, --reps launches each")
    ap.add_argument("--reps", type=int, default=100)
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the solver runs on one GPU; multi-GPU sharding (latitude "
                                   "bands + halo exchange) is designed but not implemented",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1210_1878_amd as P
    from gen import orca

    assert torch.cuda.is_available(), "bench.py needs a ROCm device"
    dev = torch.device("cuda:0")
    if args.batch_only:
        print(json.dumps({"batch_only": True, "batched": bench_batch(P, torch, dev, log)}), flush=True)
        return
    if args.serve_only:
        out = {"serve_only": True, "horizon_s": args.serve_horizon,
               "served": bench_serve(P, torch, dev, log, horizon_s=args.serve_horizon,
                                     solo_cells=args.serve_solo_cells,
                                     budget_frac=args.serve_budget_frac),
               "served_coupled_time_steps": bench_serve(
                   P, torch, dev, lambda m: log("coupled " + m), loads=(0.8,), coupled=True,
                   horizon_s=args.serve_horizon, solo_cells=args.serve_solo_cells,
                   budget_frac=args.serve_budget_frac)}
        print(json.dumps(out), flush=True)
        return
    t0 = time.perf_counter()
    p = orca.orca_problem(NX, NY, orca.CONFIG_SEED_BASE + 2)
    log(f"generated {NX}x{NY} in {time.perf_counter() - t0:.1f}s")
    A = P.Stencil5.from_problem(p)
    # the FP64 oracle's solution, for the mixed forms' error: computed on a
    # host thread while the device work goes on (the oracle releases the
    # interpreter while it runs)
    oracle_x = {}
    if not args.no_cpu and not args.kernels_only:
        import threading

        def _oracle_solution():
            import oracle
            F = oracle.ainv_setup(p, TAU)
            r = oracle.pcg(p, F, tol=TOL)
            oracle_x["x"], oracle_x["iters"] = r.x, r.iters
        ora_thread = threading.Thread(target=_oracle_solution, daemon=True)
        ora_thread.start()
    t0 = time.perf_counter()
    G = P.ainv_setup(A, TAU)
    setup_s = time.perf_counter() - t0
    log(f"ainv_setup {setup_s:.2f}s nnz_off={G.nnz_off} ({G.nnz_off / p.n:.2f}/cell)")
    # (the solver's cache plan keeps the resident set far enough below the
    # cache's size that the workspace's placement no longer matters: no probe)
    S64 = P.Solver(A, G, "fp64", device=dev, probe_placements=PLACEMENTS)
    log("fp64 placement probe (ms per iteration): "
        + ", ".join(f"{t:.4f}" for t in (S64.placement_ms or [])))
    Smx = P.Solver(A, G, "mixed", device=dev)
    for S in (S64, Smx):
        S.tune(chunk=args.chunk, use_graph=not args.no_graph, max_blocks=args.max_blocks)
    b = torch.from_numpy(p.b).to(dev)
    torch.cuda.synchronize()

    if args.kernels_only:
        src = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        ms = S64.profile_iteration(b, reps=args.reps, mode=1)
        ms32 = Smx.profile_iteration(b, reps=args.reps, mode=1)
        # the time-step passes around the solve, for the kernel trace
        from gen import orca
        faces = [torch.from_numpy(f).to(dev) for f in orca.orca_transports(p, 0, CONFIG_TS_SEED)]
        for _ in range(20):
            S64.ts_rhs(*faces)
            S64.ts_guess(faces[1], faces[3], 2.0, -1.0)
            S64.ts_eta(faces[1], faces[3], 0.5)
        torch.cuda.synchronize()
        kb = kernel_bytes(p.n, G.nnz_off, 8, S64.index_bytes, x_in_stencil(S64))
        kb32 = kernel_bytes(p.n, G.nnz_off, 4, Smx.index_bytes, x_in_stencil(Smx))
        for tag, t, byt in (("fp64", ms, kb), ("fp32", ms32, kb32)):
            log(tag + " " + ", ".join(f"{k}={t[i] * 1e3:.2f} us ({byt[k] / (t[i] * 1e-3) / 1e9:.0f} GB/s)"
                                      for i, k in enumerate(byt))
                + f", iteration={t[3] * 1e3:.2f} us")
        print(json.dumps({"kernels_only": True, "fp64_ms": ms, "fp32_ms": ms32, "bytes_fp64": kb,
                          "bytes_fp32": kb32, "n": p.n, "nnz_off": G.nnz_off,
                          "index_bytes": S64.index_bytes, "formats_fp64": S64.formats,
                          "formats_fp32": Smx.formats}), flush=True)
        return

    for _ in range(args.warmup):
        S64.solve(b, tol=TOL)
        Smx.solve_mixed(b, tol=TOL)
    torch.cuda.synchronize()

    # ---- timed region: K FP64 solves -------------------------------------
    iters = 0
    per_solve = []          # each solve returns after its result is on the host
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ts = time.perf_counter()
        r = S64.solve(b, tol=TOL)
        per_solve.append((time.perf_counter() - ts, r.iters))
        iters += r.iters
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    med_s, med_it = sorted(per_solve)[len(per_solve) // 2]
    it_s = iters / dt
    log(f"fp64: {args.steps} solves, {iters} iterations, {dt * 1e3 / args.steps:.2f} ms/solve, "
        f"{it_s:.0f} it/s, true relres {r.true_relres:.2e}")
    fp64_true = r.true_relres
    fp64_iters = r.iters

    # ---- mixed precision on the same GPU ---------------------------------
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        m = Smx.solve_mixed(b, tol=TOL, inner_tol=1e-5, max_outer=30)
    torch.cuda.synchronize()
    dtm = (time.perf_counter() - t0) / args.steps
    x64 = S64.solve(b, tol=TOL).x
    err_mx = float((m.x - x64).norm() / x64.norm())
    log(f"mixed: {dtm * 1e3:.2f} ms/solve, outer {m.outer}, inner {m.inner_total}, "
        f"true relres {m.true_relres:.2e}, |x_mixed - x_fp64|/|x_fp64| {err_mx:.2e}")
    x_mixed = m.x.cpu().numpy()
    # the same refinement with the inner direction kept across corrections
    Smx.solve_mixed(b, tol=TOL, refine="keep")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        mk = Smx.solve_mixed(b, tol=TOL, inner_tol=KEEP_SEGMENT, refine="keep")
    torch.cuda.synchronize()
    dtk = (time.perf_counter() - t0) / args.steps
    x_keep = mk.x.cpu().numpy()
    log(f"mixed, direction kept: {dtk * 1e3:.2f} ms/solve, corrections {mk.outer}, "
        f"inner {mk.inner_total}, true relres {mk.true_relres:.2e}")
    # the inner operator in FP32 too
    Sa32 = P.Solver(A, G, "mixed_a32", device=dev)
    Sa32.tune(chunk=args.chunk, use_graph=not args.no_graph, max_blocks=args.max_blocks)
    Sa32.solve_mixed(b, tol=TOL)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ma = Sa32.solve_mixed(b, tol=TOL, inner_tol=1e-5, max_outer=30)
    torch.cuda.synchronize()
    dta = (time.perf_counter() - t0) / args.steps
    Sa32.solve_mixed(b, tol=TOL, refine="keep")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        mak = Sa32.solve_mixed(b, tol=TOL, inner_tol=KEEP_SEGMENT, refine="keep")
    torch.cuda.synchronize()
    dtak = (time.perf_counter() - t0) / args.steps
    ms_a32 = Sa32.profile_iteration(b, reps=100, mode=1)
    x_a32 = ma.x.cpu().numpy()
    x_a32k = mak.x.cpu().numpy()
    log(f"mixed, FP32 operator, direction kept: {dtak * 1e3:.2f} ms/solve, corrections "
        f"{mak.outer}, inner {mak.inner_total}")
    log(f"mixed, FP32 operator: {dta * 1e3:.2f} ms/solve, outer {ma.outer}, inner {ma.inner_total}, "
        f"true relres {ma.true_relres:.2e}, inner iteration {ms_a32[3] * 1e3:.1f} us")
    Sa32.close()

    # ---- a general sparse (CSR) SPD matrix: unstructured, not a grid -------
    csr = None if args.no_csr else bench_csr(P, torch, dev, log)

    # ---- Jacobi (NEMO diagonal preconditioner) baseline on the GPU ---------
    Gj = P.ainv_setup(A, float("inf"))
    Sj = P.Solver(A, Gj, "fp64", device=dev)
    Sj.tune(chunk=args.chunk, use_graph=not args.no_graph, max_blocks=args.max_blocks)
    Sj.solve(b, tol=TOL)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rj = Sj.solve(b, tol=TOL)
    torch.cuda.synchronize()
    dtj = time.perf_counter() - t0
    log(f"jacobi: {rj.iters} iterations, {dtj * 1e3:.2f} ms/solve")

    # ---- the paper's own preconditioner: banded factor of T, q = 4 ---------
    Gb = P.fsai_band_setup(A, 4)
    Sb = P.Solver(A, Gb, "fp64", device=dev)
    Sb.tune(chunk=args.chunk, use_graph=not args.no_graph, max_blocks=args.max_blocks)
    Sb.solve(b, tol=TOL)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rb = Sb.solve(b, tol=TOL)
    torch.cuda.synchronize()
    dtb = time.perf_counter() - t0
    log(f"banded factor of T (q=4, diagonal storage): {rb.iters} iterations, {dtb * 1e3:.2f} ms/solve")

    # ---- the second Bridson class of Sec. 5: a fixed count per column of Z ---
    fixed_fill = []
    for tau_f, fill in FIXED_FILL:
        Gf = P.ainv_setup(A, tau_f, fill=fill)
        Sf = P.Solver(A, Gf, "fp64", device=dev)
        Sf.tune(chunk=args.chunk, use_graph=not args.no_graph, max_blocks=args.max_blocks)
        Sf.solve(b, tol=TOL)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rf = Sf.solve(b, tol=TOL)
        torch.cuda.synchronize()
        dtf = time.perf_counter() - t0
        fixed_fill.append({"drop_tol": tau_f, "fill": fill, "nnz_off": Gf.nnz_off,
                           "iters": rf.iters, "ms_per_solve": round(dtf * 1e3, 3),
                           "true_relres": rf.true_relres})
        log(f"fixed fill (drop_tol {tau_f}, {fill} per column): nnz_off {Gf.nnz_off} "
            f"({Gf.nnz_off / p.n:.2f}/cell), {rf.iters} iterations, {dtf * 1e3:.2f} ms/solve")
        Sf.close()
        del Gf

    # ---- autotuner on the benchmark grid (reported; the timed solves above use
    # the defaults the committed profiles describe) -------------------------
    tuned64 = None
    if not args.no_tune:
        from paper_1210_1878_amd import autotune
        t0 = time.perf_counter()
        tuned64 = autotune.tune_solver(A, G, b, "fp64", device=dev)
        log(f"autotune fp64 ({time.perf_counter() - t0:.1f}s): slice width {tuned64['slice_width']}, "
            f"blocks {tuned64['max_blocks']}, chunk {tuned64['chunk']}, "
            f"{tuned64['iteration_ms'] * 1e3:.1f} us per iteration")
        tuned64 = {"slice_width": tuned64["slice_width"], "max_blocks": tuned64["max_blocks"],
                   "chunk": tuned64["chunk"], "iteration_us": round(tuned64["iteration_ms"] * 1e3, 2),
                   "table_us": [[w, mb, round(ms * 1e3, 2)] for w, mb, ms in tuned64["table"]],
                   "chunk_ms_per_solve": [[c, round(ms, 2)] for c, ms in tuned64["chunks"]]}

    # ---- the time step around the solve (eq. (1), eq. (8), first guess) ----
    tstep = None if args.no_timestep else bench_timestep(P, torch, S64, p, log)

    # ---- roofline of the dominant kernel (HIP events on the solver stream) --
    ms = S64.profile_iteration(b, reps=100, mode=1)
    ms32 = Smx.profile_iteration(b, reps=100, mode=1)
    kb = kernel_bytes(p.n, G.nnz_off, 8, S64.index_bytes, x_in_stencil(S64))
    kb32 = kernel_bytes(p.n, G.nnz_off, 4, Smx.index_bytes, x_in_stencil(Smx))
    sb = survey_bytes(p.n, G.nnz_off, x_in_stencil(S64))
    names = list(kb)
    gbs = {k: kb[k] / (ms[i] * 1e-3) / 1e9 for i, k in enumerate(names)}
    gbs32 = {k: kb32[k] / (ms32[i] * 1e-3) / 1e9 for i, k in enumerate(names)}
    dom = max(range(3), key=lambda i: ms[i])
    log("fp64 kernels ms: " + ", ".join(f"{k}={ms[i]:.4f} ({gbs[k]:.0f} GB/s)" for i, k in enumerate(names))
        + f", iteration={ms[3]:.4f}")
    log("fp32 kernels ms: " + ", ".join(f"{k}={ms32[i]:.4f} ({gbs32[k]:.0f} GB/s)" for i, k in enumerate(names))
        + f", iteration={ms32[3]:.4f}")
    b_iter = sum(kb.values())
    # land cells are identity rows with no Z entries: the same per-iteration
    # bytes counted over ocean cells only (Z entries are all ocean)
    n_ocean = int(p.ocean.sum())
    b_iter_ocean = sum(kernel_bytes(n_ocean, G.nnz_off, 8, S64.index_bytes, x_in_stencil(S64)).values())
    b_iter32 = sum(kb32.values())
    it_time = ms[3] * 1e-3
    kname = kernel_names(8, S64.formats)[names[dom]]
    traffic, tnote = measured_traffic(kname)
    rp_us = traced_us(kname)
    dom_bytes = sb[names[dom]]
    roof = {"bound": "hbm", "kernel": kname,
            "achieved": round(dom_bytes / (ms[dom] * 1e-3) / 1e9, 1), "peak": PEAK_HBM_GBS,
            "unit": "GB/s", "frac": round(dom_bytes / (ms[dom] * 1e-3) / 1e9 / PEAK_HBM_GBS, 4),
            "traffic": traffic,
            "traffic_note": "rocprofv3 FETCH_SIZE and WRITE_SIZE per launch, each scaled by its "
                            "reading on a plain device copy: bytes the L2 fetched from and wrote "
                            "to memory, including reads served by the 256 MiB memory-side cache, "
                            "so an upper bound of the HBM traffic (" + tnote + ")",
            "bytes_per_launch": dom_bytes,
            "bytes_model": ("method steps alpha, r' = r - alpha q and ||r||^2 (24 n; the x axpy "
                            "is done by the stencil) and D^-1 Z^T r (24 n + 12 nnz_off)"
                            if x_in_stencil(S64) else
                            "method steps alpha + axpys + ||r||^2 (48 n) and D^-1 Z^T r "
                            "(24 n + 12 nnz_off)") + ", FP64 values and int32 indices",
            "ms_per_launch": ms[dom],
            "rocprof_us_per_launch": rp_us,
            "frac_rocprof": None if rp_us is None else round(dom_bytes / (rp_us * 1e-6) / 1e9 / PEAK_HBM_GBS, 4),
            "kernel_own_bytes_per_launch": kb[names[dom]],
            "frac_kernel_own_bytes": round(gbs[names[dom]] / PEAK_HBM_GBS, 4),
            "per_iteration": {"bytes": sb["iteration"], "us": round(ms[3] * 1e3, 2),
                              "frac": round(sb["iteration"] / it_time / 1e9 / PEAK_HBM_GBS, 4),
                              "frac_whole_solve": round(sb["iteration"] * it_s / 1e9 / PEAK_HBM_GBS, 4),
                              "model": "152 n + 24 nnz_off bytes per FP64 iteration"}}

    batched = None if args.no_batch else bench_batch(P, torch, dev, log)
    served = None if args.no_serve else bench_serve(P, torch, dev, log, compare_fp64=True,
                                                    horizon_s=args.serve_horizon,
                                                    solo_cells=args.serve_solo_cells,
                                                    budget_frac=args.serve_budget_frac)
    served_coupled = None if args.no_serve or args.no_timestep else bench_serve(
        P, torch, dev, lambda m: log("coupled " + m), loads=(0.8,), coupled=True,
        horizon_s=args.serve_horizon, solo_cells=args.serve_solo_cells,
        budget_frac=args.serve_budget_frac)

    cpu = None
    err_ora = err_a32_ora = err_keep_ora = err_a32k_ora = None
    if not args.no_cpu:
        ora_thread.join()
        xo = oracle_x["x"]
        err_ora = float(np.linalg.norm(x_mixed - xo) / np.linalg.norm(xo))
        err_a32_ora = float(np.linalg.norm(x_a32 - xo) / np.linalg.norm(xo))
        err_keep_ora = float(np.linalg.norm(x_keep - xo) / np.linalg.norm(xo))
        err_a32k_ora = float(np.linalg.norm(x_a32k - xo) / np.linalg.norm(xo))
        log(f"mixed vs the FP64 oracle's solution ({oracle_x['iters']} iterations): "
            f"{err_ora:.2e}; with the FP32 operator {err_a32_ora:.2e}")
        log(f"cpu baseline (oracle, ~{args.cpu_seconds:.0f}s)")
        cpu = cpu_baseline(p, args.cpu_seconds)
        log(f"cpu: {cpu['value']:.2f} it/s")

    out = {
        "metric": METRIC, "value": round(it_s, 1), "unit": "iter/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(dt * 1e3 / args.steps, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "ORCA025-shaped 1442x1021 lat-lon grid (lat -78..90, EW periodic, "
                               "35% land, seeded depth 500-5500 m), AINV drop tol 0.05, FP64 "
                               "PCG to relres 1e-10 from x0=0",
                   "nx": NX, "ny": NY, "n": p.n, "nnz_off": G.nnz_off, "index_bytes": S64.index_bytes, "formats": {"fp64": S64.formats, "mixed": Smx.formats}, "tol": TOL,
                   "drop_tol": TAU, "iters_per_solve": fp64_iters, "chunk": args.chunk,
                   "graph": not args.no_graph, "max_blocks": args.max_blocks or "default: fp64 1280, mixed 1536",
                   "slice_width": {"fp64": S64.slice_width or 24, "mixed": Smx.slice_width or 24}},
        "fp64": {"iters": fp64_iters, "ms_per_solve": round(dt * 1e3 / args.steps, 3),
                 "true_relres": fp64_true, "model_bytes_per_iter": b_iter,
                 "model_gbs_per_iter_kernels": round(b_iter / it_time / 1e9, 1),
                 "model_gbs_whole_solve": round(b_iter * it_s / 1e9, 1),
                 "placement_probe_ms_per_iter": [round(t, 5) for t in (S64.placement_ms or [])],
                 "ms_per_solve_median": round(med_s * 1e3, 3),
                 "it_s_median_solve": round(med_it / med_s, 1),
                 "ocean_cells": n_ocean,
                 "model_bytes_per_iter_ocean_only": b_iter_ocean,
                 "model_gbs_whole_solve_ocean_only": round(b_iter_ocean * it_s / 1e9, 1),
                 "kernel_ms": dict(zip(names, [round(v, 5) for v in ms[:3]])),
                 "iteration_ms": round(ms[3], 5)},
        "mixed": {"ms_per_solve": round(dtm * 1e3, 3), "outer": m.outer, "inner_iters": m.inner_total,
                  "inner_it_s": round(m.inner_total / dtm, 1), "true_relres": m.true_relres,
                  "rel_err_vs_fp64": err_mx, "rel_err_vs_oracle": err_ora,
                  "speedup_vs_fp64": round(dt / args.steps / dtm, 3),
                  "model_bytes_per_inner_iter": b_iter32,
                  "kernel_ms": dict(zip(names, [round(v, 5) for v in ms32[:3]])),
                  "iteration_ms": round(ms32[3], 5)},
        "mixed_keep_direction": {
            "refine": "inner direction kept across corrections (reliable updates), "
                      f"each inner run reducing its residual by {KEEP_SEGMENT}",
            "ms_per_solve": round(dtk * 1e3, 3), "corrections": mk.outer,
            "inner_iters": mk.inner_total, "true_relres": mk.true_relres,
            "rel_err_vs_oracle": err_keep_ora, "speedup_vs_fp64": round(dt / args.steps / dtk, 3),
            "speedup_vs_restarted": round(dtm / dtk, 3)},
        "mixed_fp32_operator": {"ms_per_solve": round(dta * 1e3, 3), "outer": ma.outer,
                                "inner_iters": ma.inner_total, "true_relres": ma.true_relres,
                                "rel_err_vs_oracle": err_a32_ora,
                                "speedup_vs_fp64": round(dt / args.steps / dta, 3),
                                "iteration_ms": round(ms_a32[3], 5),
                                "keep_direction": {"ms_per_solve": round(dtak * 1e3, 3),
                                                   "corrections": mak.outer,
                                                   "inner_iters": mak.inner_total,
                                                   "true_relres": mak.true_relres,
                                                   "rel_err_vs_oracle": err_a32k_ora,
                                                   "speedup_vs_fp64":
                                                       round(dt / args.steps / dtak, 3)}},
        "csr_unstructured": csr,
        "jacobi": {"iters": rj.iters, "ms_per_solve": round(dtj * 1e3, 3),
                   "true_relres": rj.true_relres},
        "band_factor_q4": {"iters": rb.iters, "ms_per_solve": round(dtb * 1e3, 3),
                           "true_relres": rb.true_relres, "band_q": Sb.band_q},
        "fixed_fill": fixed_fill,
        "autotune_fp64": tuned64,
        "timestep": tstep,
        "batched": batched,
        "served": served,
        "served_coupled_time_steps": served_coupled,
        "setup_s": round(setup_s, 3),
        "roofline": roof,
        # the paper's figures (Sec. 6), quoted with their hardware as context;
        # flops per iteration: the five-point product (9 n), the two sparse
        # products (2 flops per nonzero of Z in each, plus 3 n for the unit
        # diagonals and D^-1), three dot products and three axpys (12 n)
        "paper_context": {"gpu_gflops": 87.0, "gpu": "NVIDIA Tesla S2050 (Fermi), FP32, CUBLAS/CUSPARSE CSR",
                          "cpu_gflops": 1.43, "cpu": "Intel Xeon E5620, serial ANSI C, FP32",
                          "workload": "ORCA-025 1442x1021, NEMO mesh",
                          "this_fp64_gflops": round((24.0 * p.n + 4.0 * G.nnz_off) * it_s / 1e9, 1),
                          "flops_per_iter": 24 * p.n + 4 * G.nnz_off},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
