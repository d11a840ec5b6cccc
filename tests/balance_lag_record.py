"""How well a map computed from one window's measured loads fits the next window.

    python tests/balance_lag_record.py [--workload large] [--out profiles/balance_lag_large.json]

The paper measures loads during a window of steps and migrates at its end (Fig. 2,
Section VI: the last M steps of each window of R are measured).  With a moving
hotspot the map is then used on a window whose loads have moved on.  This record
takes the exact per-step work loads of a workload (the oracle's closed form, the
same values the library measures bit for bit), runs the workload's balancer at
every rebalance point from the loads of the last M steps of the window (R = 10),
and reports, for the window each map is then used on:
  lambda_fit     max slot load / mean slot load of the map on the loads it was
                 computed from (what the balancer achieved);
  lambda_next    the same on the next window's loads (the map in force);
  lambda_star    max(1, S * max chunk load / total), the bound of any chunk map,
                 on the next window's loads;
  lambda_block   the static block map on the next window's loads;
  migrations     chunks moved at that rebalance.
Means over the rebalance points, for M = 1, 4, R (all steps) and R = 5, 10, 20, with
the workload's own strategy and, for comparison, GreedyLB at every point and the
Greedy-then-RefineSwap policy of Experiment C.
Host only; test infrastructure (it imports the oracle).
"""
from __future__ import annotations

import argparse
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from paper_1310_4218_amd import workloads as W  # noqa: E402


def lam(w, m, S):
    L = np.bincount(m, weights=w, minlength=S)
    return float(L.max() / (w.sum() / S))


def step_loads(wl, T):
    """Exact work loads of every step (T x C)."""
    out = np.empty((T, wl.nchunks))
    for t in range(T):
        k = oracle.kfield(wl.nx, wl.ny, wl.hot, wl.t0 + t, wl.sigma, wl.kmin, wl.kmax)
        out[t] = oracle.chunk_work(k, wl.nz, wl.xsplit, wl.ysplit, wl.alpha_work) * wl.nfields
    return out


def simulate(wl, loads, R, M, strategy):
    S, C = wl.nslots, wl.nchunks
    T = loads.shape[0]
    m = oracle.block_map(C, S)
    block = m.copy()
    rows = []
    first = True
    for t in range(R, T - R + 1, R):           # rebalance points R, 2R, ... with a next window
        meas = loads[t - M:t].sum(axis=0)
        old = m
        if strategy == "greedy" or (strategy == "greedy_then_refineswap" and first):
            m = oracle.greedy(meas, S)
        elif strategy == "refine":
            m = oracle.refine(meas, m, S, wl.threshold)
        else:
            m = oracle.refineswap(meas, m, S, wl.threshold)
        first = False
        nxt = loads[t:t + R].sum(axis=0)
        rows.append(dict(step=t, lambda_fit=lam(meas, m, S), lambda_next=lam(nxt, m, S),
                         lambda_star=max(1.0, S * nxt.max() / nxt.sum()), lambda_block=lam(nxt, block, S),
                         migrations=int((m != old).sum())))
    keys = ("lambda_fit", "lambda_next", "lambda_star", "lambda_block", "migrations")
    return {k: float(np.mean([r[k] for r in rows])) for k in keys} | dict(rebalances=len(rows))


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawTextHelpFormatter)
    ap.add_argument("--workload", default="large")
    ap.add_argument("--steps", type=int, default=None, help="steps to model (default: the workload's)")
    ap.add_argument("--out", default=None)
    args = ap.parse_args(argv)
    wl = W.get(args.workload)
    T = args.steps or wl.steps
    loads = step_loads(wl, T)
    res = dict(workload=wl.name, slots=wl.nslots, chunks=wl.nchunks, steps=T, strategy=wl.strategy,
               threshold=wl.threshold, command="python tests/balance_lag_record.py --workload " + args.workload,
               runs=[])
    strategies = [wl.strategy] + [s for s in ("greedy", "greedy_then_refineswap") if s != wl.strategy]
    for strategy in strategies:
        for R in (5, 10, 20):
            for M in sorted({1, 4, R}):
                if M > R:
                    continue
                r = simulate(wl, loads, R, M, strategy)
                r.update(R=R, M=M, strategy=strategy)
                res["runs"].append(r)
                print(json.dumps(r), flush=True)
    out = args.out or os.path.join(ROOT, "profiles", f"balance_lag_{args.workload}.json")
    with open(out, "w") as f:
        json.dump(res, f, indent=1)
    print("wrote", out)


if __name__ == "__main__":
    main()
