"""Benchmark: grid point-updates/s and max/avg slot-load ratio, balanced vs plain, 1 GPU.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload moving]

A step is one time step of the whole hot path on the synthetic workload: the
cost field, the 7-point update, the column physics, the per-chunk load
measurement and the FP64 checksum, all in the library's HIP kernels; every
R steps (R = 10 for the default workload) the loads of the window are read
back and GreedyLB remaps the chunks onto the slots (the paper's migration
point, Section VI).  Two paths are timed on the same inputs:
  balanced: one persistent launch per step (replayed from a HIP graph of R
            steps), cost-ordered per-slot queues, measurement + rebalance every
            R steps, all inside the timed region;
  plain:    one launch per chunk in chunk-id order, no balancing.
``value`` is the balanced path's point-updates/s (cells x steps / wall time).
The default workload is the 256x256x64 grid with 64 equal chunks and a hotspot
moving one cell per step (k in 1..200, sigma 24), balanced onto 256 slots.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("kernels.hip", "lbgrid_internal.h"):
        with open(os.path.join(ROOT, "paper_1310_4218_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload: str):
    """HBM bytes per launch of the persistent kernel from committed rocprofv3 counter
    summaries, if they were taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("kernel_source_hash") != kernel_source_hash():
        return None
    return t.get("hbm_bytes_per_launch")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def run_balanced(Grid, wl, steps, warmup, R, strategy, threshold, torch):
    import numpy as np

    g = Grid(wl, graph_steps=R)
    stream = g.stream

    def window(n, events=None):
        if events is not None:
            events[0].record(stream)
        g.step(n, "persistent")
        if events is not None:
            events[1].record(stream)
        loads = g.measure("work")            # synchronizes: the paper's measurement point
        lam = g.rebalance(strategy, threshold, None)
        return loads, lam

    done = 0
    while done < warmup:                     # warm-up windows (graph capture happens here)
        n = min(R, warmup - done)
        window(n)
        done += n
    g.measure("work")                        # fresh window, fresh busy counters
    torch.cuda.synchronize()
    evs = []
    lam_win, loads_win = [], []
    t0 = time.perf_counter()
    done = 0
    while done < steps:
        n = min(R, steps - done)
        ev = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
        busy_before = None
        loads, (m, nmig, (lam_before, lam_after)) = window(n, ev)
        evs.append((ev, n))
        lam_win.append((lam_before, lam_after, nmig))
        loads_win.append(loads)
        done += n
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kernel_s = sum(e[0].elapsed_time(e[1]) for e, _ in evs) / 1e3
    # workgroup balance of the persistent kernel over one extra measured window
    g.measure("work")
    g.step(R, "persistent")
    busy = g.wg_busy()
    w_last = g.measure("work")
    st = g.stats()
    g.close()
    return dict(wall=wall, kernel_s=kernel_s, lam=lam_win, loads=loads_win, busy=busy,
                w_last=w_last, stats=st)


def run_plain(Grid, wl, steps, warmup, torch):
    g = Grid(wl)
    g.step(warmup, "plain")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.step(steps, "plain")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    g.close()
    return dict(wall=wall)


def cpu_baseline(wl, budget_s):
    import oracle

    t = time.perf_counter()
    oracle.run(wl, nsteps=1)
    one = max(time.perf_counter() - t, 1e-6)
    n = max(1, min(wl.steps, int(budget_s / one)))
    t = time.perf_counter()
    oracle.run(wl, nsteps=n)
    dt = time.perf_counter() - t
    return dict(value=wl.ncells * n / dt, unit="point-updates/s", cores=1, kind="oracle",
                sample=f"{n} steps of the {wl.name} workload from the seeded field "
                       f"(single-threaded FP64 C oracle)")


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawTextHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="moving")
    ap.add_argument("--plain-steps", type=int, default=None)
    ap.add_argument("--cpu-budget", type=float, default=12.0, help="seconds of oracle work")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    args = ap.parse_args(argv)

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); this build has no "
              "multi-GPU path", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    from paper_1310_4218_amd import workloads as W
    from paper_1310_4218_amd.grid import Grid

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    wl = W.get(args.workload)
    R = wl.rebalance_every or 10
    S = wl.nslots
    log(f"bench: {wl.name} steps={args.steps} warmup={args.warmup} R={R} S={S}")

    bal = run_balanced(Grid, wl, args.steps, args.warmup, R, wl.strategy, wl.threshold, torch)
    log(f"balanced: {bal['wall'] * 1e3 / args.steps:.4f} ms/step, kernel {bal['kernel_s'] * 1e3 / args.steps:.4f} ms/step")
    plain = None
    if not args.no_plain:
        ps = args.plain_steps or args.steps
        plain = run_plain(Grid, wl, ps, max(1, args.warmup // 2), torch)
        plain["steps"] = ps
        log(f"plain: {plain['wall'] * 1e3 / ps:.4f} ms/step")

    value = wl.ncells * args.steps / bal["wall"]
    # imbalance over the timed windows (the first window ran on the map of the warm-up)
    import oracle  # noqa: F401  (only for the CPU baseline below)
    from paper_1310_4218_amd._abi import balance_host  # host balancer = the library's own

    lam_bal = float(np.mean([l[0] for l in bal["lam"]]))
    block = np.array([(c * S) // wl.nchunks if wl.nchunks >= S else c for c in range(wl.nchunks)])

    def lam_of(w, m):
        L = np.bincount(m, weights=w, minlength=S)
        return float(L.max() / (w.sum() / S))

    lam_plain = float(np.mean([lam_of(w, block) for w in bal["loads"]]))
    lam_star = float(np.mean([max(1.0, S * w.max() / w.sum()) for w in bal["loads"]]))
    busy = bal["busy"]
    lam_wg = float(busy.max() / busy.mean()) if busy.mean() > 0 else None

    elem = 8 if False else 4
    bytes_per_step = 2 * elem * wl.ncells * wl.nfields
    kernel_step_s = bal["kernel_s"] / args.steps
    achieved = bytes_per_step / kernel_step_s / 1e9
    traffic = measured_traffic(args.workload)

    out = {
        "metric": "grid point-updates/s and max/avg chunk-load ratio, balanced vs plain, 1 MI355X",
        "value": value,
        "unit": "point-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": bal["wall"] * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wl.name, "grid": [wl.nx, wl.ny, wl.nz], "chunks": wl.nchunks,
                   "slots": S, "rebalance_every": R, "strategy": wl.strategy,
                   "parallelism": "single-gpu"},
        "balanced_vs_plain": {
            "balanced_point_updates_per_s": value,
            "plain_point_updates_per_s": (wl.ncells * plain["steps"] / plain["wall"]) if plain else None,
            "speedup": (value / (wl.ncells * plain["steps"] / plain["wall"])) if plain else None,
            "lambda_balanced": lam_bal,
            "lambda_plain": lam_plain,
            "lambda_star": lam_star,
            "lambda_wg": lam_wg,
            "migrations_per_rebalance": float(np.mean([l[2] for l in bal["lam"]])),
        },
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "kernel": "k_persistent<float,4,0>",
            "kernel_us_per_step_events": kernel_step_s * 1e6,
        },
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(wl, args.cpu_budget)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
