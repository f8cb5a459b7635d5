"""Autotuner: picks the launch and layout settings of a grid by timing them.

For one grid (`tune_solver`): the sliced-ELL target width (how many entry
steps a slice may take before its rows get more lanes), the number of
workgroups per kernel and the iterations per graph chunk.  Width and
workgroup count are timed as whole PCG iterations replayed in a solve's cache
state (`Solver.profile_iteration`, mode 1); the chunk, which trades the
host's polling against iterations run past convergence, by whole solves.

For an ensemble (`tune_batch`): the target width of its solvers and the
batch's iterations per chunk, timed as whole batched solves of the ensemble.

Every candidate is the same method; settings change only speed and the
rounding order inside a row (a different width).  Results are plain dicts so
that a caller can store and reuse them.
"""
from __future__ import annotations

import time

from .api import Batch, Solver, workspace_size

WIDTHS = (8, 12, 16, 24, 32)
CHUNKS = (16, 32, 64)


def _blocks_for(precision):
    return (1024, 1280, 1536, 1792, 2048) if precision == "mixed" else (1024, 1280, 1536, 2048)


def tune_solver(A, F, b, precision="fp64", widths=WIDTHS, blocks=None, chunks=CHUNKS,
                reps=20, tol=1e-10, device=None, log=None):
    """Best (slice_width, max_blocks, chunk) for this grid, with every timing.

    Returns {"slice_width", "max_blocks", "chunk", "iteration_ms": best whole
    iteration, "table": [(width, blocks, ms per iteration)], "chunks":
    [(chunk, ms per solve)]}."""
    import torch
    blocks = _blocks_for(precision) if blocks is None else blocks
    table = []
    best = None
    # every candidate is carved from one buffer, at one address: an FP64
    # iteration's time depends on where its workspace sits in memory, which
    # would otherwise differ from candidate to candidate
    buf = torch.empty(max(workspace_size(A, F, precision, w) for w in widths),
                      dtype=torch.uint8, device=torch.device("cuda" if device is None else device))
    for w in widths:
        S = Solver(A, F, precision, device=device, slice_width=w, buffer=buf)
        for mb in blocks:
            S.tune(max_blocks=mb)
            S.profile_iteration(b, reps=2, mode=1)          # capture, first touch
            ms = S.profile_iteration(b, reps=reps, mode=1)[3]
            table.append((w, mb, ms))
            if log:
                log(f"width {w} blocks {mb}: {ms * 1e3:.1f} us per iteration")
            if best is None or ms < best[2]:
                best = (w, mb, ms)
        S.close()
        torch.cuda.synchronize()     # nothing may still use buf when it is rebuilt
    w, mb, it_ms = best
    S = Solver(A, F, precision, device=device, slice_width=w, buffer=buf)
    solve = S.solve if precision == "fp64" else S.solve_mixed
    timings = []
    for c in chunks:
        S.tune(chunk=c, max_blocks=mb)
        solve(b, tol=tol)                                    # capture at this chunk
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(2):
            solve(b, tol=tol)
        torch.cuda.synchronize()
        timings.append((c, (time.perf_counter() - t0) / 2 * 1e3))
        if log:
            log(f"chunk {c}: {timings[-1][1]:.2f} ms per solve")
    S.close()
    chunk = min(timings, key=lambda t: t[1])[0]
    return {"slice_width": w, "max_blocks": mb, "chunk": chunk, "iteration_ms": it_ms,
            "table": table, "chunks": timings}


def tune_batch(make_items, widths=(8, 16, 32), chunks=(8, 16, 32), tol=1e-10, log=None,
               refine="restart"):
    """Best (slice_width, chunk) for an ensemble.

    make_items(width) returns [(solver, B)] (a mixed solver built with that
    slice width and its right-hand sides [nrhs, n]); each candidate solves
    the whole ensemble in one batch with the given refinement.  Returns
    {"slice_width", "chunk", "table": [(width, chunk, ms)]}."""
    import torch
    table = []
    for w in widths:
        items = make_items(w)
        for c in chunks:
            Bt = Batch(max_slots=len(items), chunk=c)
            for S, B in items:
                Bt.add(S, B, tol=tol, refine=refine)
            Bt.solve()                                        # capture, first touch
            for S, B in items:
                Bt.add(S, B, tol=tol, refine=refine)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            Bt.solve()
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3
            table.append((w, c, ms))
            if log:
                log(f"batch width {w} chunk {c}: {ms:.1f} ms")
            Bt.close()
        for S, _ in items:
            S.close()
    w, c, _ = min(table, key=lambda t: t[2])
    return {"slice_width": w, "chunk": c, "table": table}
