"""Load-measurement study: which per-chunk load source gives the best chunk map?

    python -m paper_1310_4218_amd.study --workload moving [--windows 3]

Section V of the paper finds GPU load measurement reliable only when kernels
run one at a time (synchronous launches), and unreliable under concurrent
kernels.  This study compares three sources of per-chunk load on the same
window of steps:
  work          deterministic work units, nz*(alpha + k) per column;
  time/plain    in-kernel wall-clock ticks with one launch per chunk (chunks
                run one after another: the paper's synchronous mode);
  time/persist  in-kernel wall-clock ticks inside the persistent launch, where
                all chunks run concurrently and share the GPU.
For each source the chunks are mapped with GreedyLB, and the map is judged
  (a) by its imbalance under the work loads (lambda_work), and
  (b) by the measured time of persistent steps run with that map and with
      stealing off, so that the map alone decides the balance.
Also reported: Spearman rank correlation of each time source with the work
loads.  Prints one JSON line per window; with --out, writes them all as one JSON
record (the workload, slots, and per window the rank correlations and, per
source, the map's imbalance and timed step).
"""
from __future__ import annotations

import argparse
import json
import sys

import numpy as np


def spearman(a, b) -> float:
    ra = np.argsort(np.argsort(a)).astype(float)
    rb = np.argsort(np.argsort(b)).astype(float)
    ra -= ra.mean()
    rb -= rb.mean()
    d = np.sqrt((ra ** 2).sum() * (rb ** 2).sum())
    return float((ra * rb).sum() / d) if d > 0 else 1.0


def lam(w, m, S) -> float:
    L = np.bincount(m, weights=w, minlength=S)
    return float(L.max() / (w.sum() / S))


def run(wl, windows=3, R=None, steps_timed=10, log=print, keep_loads=False):
    """One result per window (see the module docstring); with keep_loads the three
    load vectors and the three maps are kept in it as well (not in the JSON lines)."""
    import torch

    from ._abi import balance_host
    from .grid import Grid

    R = R or wl.rebalance_every or 10
    S = wl.nslots
    out = []
    t = 0
    for win in range(windows):
        # the same window of steps measured three ways; costs depend only on the hotspot
        # positions (time t0 + t), not on the field values, so each context starts from
        # the seeded field at time t0 + t
        start = dict(t0=wl.t0 + t)
        g_plain = Grid(wl.replace(**start))
        g_plain.step(R, "plain")
        w_plain = g_plain.measure("work", reset=False)
        t_plain = g_plain.measure("time")
        g_plain.close()
        g_pers = Grid(wl.replace(**start))
        g_pers.step(R, "persistent")
        w_pers = g_pers.measure("work", reset=False)
        t_pers = g_pers.measure("time")
        g_pers.close()
        assert np.array_equal(w_plain, w_pers)
        w = w_pers
        maps = {}
        for name, loads in (("work", w), ("time/plain", t_plain), ("time/persist", t_pers)):
            maps[name], _ = balance_host(loads, S, "greedy")
        res = dict(window=win, steps=[t, t + R],
                   spearman_time_plain=spearman(t_plain, w),
                   spearman_time_persist=spearman(t_pers, w), maps={})
        # time the next window under each map, stealing off
        for name, m in maps.items():
            g = Grid(wl.replace(t0=wl.t0 + t + R), steal=0)
            g.set_map(m, w)
            g.step(2, "persistent")
            s = g.stream
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record(s)
            g.step(steps_timed, "persistent")
            e1.record(s)
            torch.cuda.synchronize()
            us = e0.elapsed_time(e1) * 1e3 / steps_timed
            g.close()
            res["maps"][name] = dict(lambda_work=lam(w, m, S), us_per_step=us)
        log(json.dumps(res))
        if keep_loads:
            res["loads"] = {"work": w, "time/plain": t_plain, "time/persist": t_pers}
            res["map_arrays"] = maps
        out.append(res)
        t += R
    return out


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawTextHelpFormatter)
    ap.add_argument("--workload", default="moving")
    ap.add_argument("--windows", type=int, default=3)
    ap.add_argument("--slots", type=int, default=None, help="override S")
    ap.add_argument("--out", default=None, help="write the record to this JSON file")
    args = ap.parse_args(argv)
    from . import workloads as W

    wl = W.get(args.workload)
    if args.slots:
        wl = wl.replace(nslots=args.slots)
    res = run(wl, args.windows, log=lambda s: print(s, flush=True))
    if args.out:
        with open(args.out, "w") as f:
            json.dump(dict(workload=wl.name, slots=wl.nslots, chunks=wl.nchunks,
                           command="python -m paper_1310_4218_amd.study " + " ".join(argv or sys.argv[1:]),
                           windows=res), f, indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(main())
