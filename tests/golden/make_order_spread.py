"""Write order_spread_1442x1021.json: how far rounding order alone moves
Algorithm 1 on the 1442x1021 ORCA025-shaped problem.

Calls only the oracle: its default build and its evaluation-order builds
(reversed or blocked inner-product sums, fused multiply-adds; oracle.c), on
the same operator, factor and right-hand side.  For each factor it records
every build's stopping iteration at tol 1e-10 and, at K = 12, 20, 30, 40
iterations and at the natural stop, the largest relative distance of a
build's iterate from the default build's.  The device tests take their
parity bars from these numbers.

    python tests/golden/make_order_spread.py        (about 5 minutes, 5 threads)
"""
import json
import os
import sys
from concurrent.futures import ThreadPoolExecutor

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from gen import orca  # noqa: E402

KS = [12, 20, 30, 40]
FACTORS = {"threshold_tau0.05": dict(tau=0.05, fill=None),
           "fixed_fill8_tau0.01": dict(tau=0.01, fill=8)}


def main():
    oracle.build(force=False)
    p = orca.orca_problem(1442, 1021, orca.CONFIG_SEED_BASE + 2)
    builds = [None] + list(oracle.VARIANTS)
    out = {"grid": "1442x1021", "seed": orca.CONFIG_SEED_BASE + 2, "tol": 1e-10,
           "builds": ["default"] + list(oracle.VARIANTS), "factors": {}}
    for label, fa in FACTORS.items():
        F = oracle.ainv_setup(p, fa["tau"], fill=fa["fill"])

        def run(v):
            xs = {K: oracle.pcg(p, F, tol=0.0, maxit=K, variant=v).x for K in KS}
            nat = oracle.pcg(p, F, tol=1e-10, variant=v)
            return v, xs, nat

        with ThreadPoolExecutor(len(builds)) as ex:
            res = {v: (xs, nat) for v, xs, nat in ex.map(run, builds)}
        ref_xs, ref_nat = res[None]
        iters = {("default" if v is None else v): int(res[v][1].iters) for v in builds}

        def spread(get):
            r = get(None)
            return max(float(np.linalg.norm(get(v) - r) / np.linalg.norm(r)) for v in builds[1:])

        out["factors"][label] = {
            "drop_tol": fa["tau"], "fill": fa["fill"], "nnz_off": F.nnz_off,
            "stop_iters": iters,
            "stop_window": [min(iters.values()), max(iters.values())],
            "iterate_spread": {str(K): spread(lambda v, K=K: res[v][0][K]) for K in KS},
            "solution_spread_at_stop": spread(lambda v: res[v][1].x),
        }
        print(label, json.dumps(out["factors"][label]), flush=True)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "order_spread_1442x1021.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()
