"""Autotuner for the launch shape of the persistent step.

    python -m paper_1310_4218_amd.autotune --workload moving [--precision fp32]

Searches the launch parameters that do not change the method (launch form
item_grid, steps per launch fuse_steps, pipeline march / stage_rows, tile_x,
tile_y, nqueues, wg_per_queue, queue order and hot_cut, item_split,
tail_split, item_alpha, xcd_group, lane_levels), keeping
everything that defines the problem fixed (grid, chunks, hotspots, number of
balancer slots S).  Each candidate: a fresh context run in windows of R steps
with a load measurement and a rebalance after each window, as the benchmark
runs; the step windows after the warm-up are timed with HIP events on the
context's stream.
Search is coordinate descent from the library defaults (two sweeps over the
parameters).  The chosen configuration must give fields bit-identical to the
library defaults after the same steps, otherwise it is rejected.

Results are cached in ``tuned.json`` next to this file, keyed by GPU
architecture, workload name and precision; ``tuned_params`` reads them.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE = os.path.join(HERE, "tuned.json")

SPACE = {
    "item_grid": [0, 1],          # 1: one workgroup per item (needs march > 0)
    "fuse_steps": [0, 2, 3],      # 2, 3: steps per launch (needs item_grid 1)
    "march": [0, 2, 4, 8],        # > 0: column-march pipeline, rows in flight
    "queue_order": [0, 1],        # 1: hot items longest first, the rest by position
    "hot_cut": [200, 120, 150, 300, 500],   # queue_order 1: hot above this % of the mean
    "tile_x": [8, 16, 32, 64],
    "tile_y": [2, 4, 8, 12, 16, 24, 32, 40, 48, 64],
    "nqueues": [1, 8, 32, 256],
    "wg_per_queue": [0],          # 0: fill the device (resident workgroups / queues)
    "item_split": [0, 1, 2, 3, 4, 5, 6, 8],
    "stage_rows": [-1, -4, -8, 2, 4, 6, 8],   # -1, -4, -8: register pipeline 2/4/8 rows deep;
                                              # n > 0: direct-to-LDS batches of n rows
    "tail_split": [0, 2, 4, 8],
    "item_alpha": [-1, 8, 4, 2, 1, 0],  # -1: items sized with the balancer's alpha_work
    "xcd_group": [0, 4, 8],       # > 1: runs of this many neighbouring items per XCD
    "lane_levels": [0, 5],        # 5: five levels per thread in the two-step launch
}


def _key(arch: str, workload: str, precision: str) -> str:
    return f"{arch}/{workload}/{precision}"


def tuned_params(workload_name: str, precision: str = "fp32", arch: str = None,
                 physics: str = "pointwise") -> dict:
    """Cached launch parameters for a workload, or {} when none were tuned.  FP32
    with Kahan summation has the FP32 data layout and kernels; without an entry
    of its own it takes the FP32 one.  physics "vertical" takes an entry of its
    own (key suffix /vertical) where there is one, else the pointwise one."""
    if not os.path.exists(CACHE):
        return {}
    with open(CACHE) as f:
        cache = json.load(f)
    if arch is None:
        arch = "gfx950"
    entry = None
    precs = (precision, "fp32") if precision in ("fp32_kahan", "kahan") else (precision,)
    suffixes = ("/vertical", "") if physics == "vertical" else ("",)
    for suf in suffixes:
        for pr in precs:
            entry = cache.get(_key(arch, workload_name, pr) + suf)
            if entry is not None:
                break
        if entry is not None:
            break
    return dict((entry or {}).get("params", {}))


def _feasible(wl, p: dict) -> bool:
    from . import _abi

    try:
        cfg, keep = _abi.config_from_workload(wl, **p)
        _abi.query(cfg)
        return True
    except Exception:
        return False


def measure(wl, params: dict, precision: str, steps: int, warm: int, torch):
    """Microseconds per persistent step for one candidate, plus its final field.

    The candidate runs as the benchmark does: windows of R steps (one graph
    replay), each followed by a load measurement and a rebalance with the
    workload's balancer, so that every window starts from a map and items cut
    from the previous window's loads.  Only the step windows are timed (HIP
    events on the context's stream)."""
    from .grid import Grid

    R = wl.rebalance_every or 10
    g = Grid(wl, precision=precision, graph_steps=R, **params)
    for _ in range(max(1, -(-warm // R))):
        g.step(R, "persistent_eager")
        g.measure("work")
        g.rebalance(wl.strategy, wl.threshold)
    evs = []
    for _ in range(max(1, -(-steps // R))):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(g.stream)
        g.step(R, "persistent_eager")
        e1.record(g.stream)
        evs.append((e0, e1))
        g.measure("work")
        g.rebalance(wl.strategy, wl.threshold)
    torch.cuda.synchronize()
    us = sum(a.elapsed_time(b) for a, b in evs) * 1e3 / (len(evs) * R)
    field = g.field()
    g.close()
    return us, field


def tune(wl, precision: str = "fp32", steps: int = 50, warm: int = 20, log=print,
         seeds=(), from_defaults: bool = True) -> dict:
    """Coordinate descent (two sweeps over SPACE) from the library defaults and
    from every extra starting point in `seeds`; the best candidate whose fields
    are bit-identical to the defaults' wins."""
    import torch

    base = {}
    t_base, f_base = measure(wl, base, precision, steps, warm, torch)
    log(f"defaults: {t_base:.2f} us/step")
    tried = {json.dumps(base, sort_keys=True): t_base}

    def descend(start: dict, t_start: float):
        best, best_t = dict(start), t_start
        for sweep in range(2):
            for name, values in SPACE.items():
                for v in values:
                    cand = dict(best)
                    cand[name] = v
                    key = json.dumps(cand, sort_keys=True)
                    if key in tried:
                        if tried[key] < best_t:
                            best, best_t = cand, tried[key]
                        continue
                    if not _feasible(wl, cand):
                        continue
                    try:
                        t, f = measure(wl, cand, precision, steps, warm, torch)
                    except Exception as e:  # a shape the library rejects at init
                        log(f"  {cand}: rejected ({e})")
                        tried[key] = float("inf")
                        continue
                    same = bool(torch.equal(f, f_base))
                    tried[key] = t if same else float("inf")
                    log(f"  {cand}: {t:.2f} us/step{'' if same else '  FIELDS DIFFER -> rejected'}")
                    if same and t < best_t:
                        best, best_t = cand, t
        return best, best_t

    best, best_t = descend(base, t_base) if from_defaults else (base, t_base)
    for seed in seeds:
        seed = {k: v for k, v in seed.items() if k in SPACE}
        key = json.dumps(seed, sort_keys=True)
        if key not in tried:
            if not _feasible(wl, seed):
                continue
            t, f = measure(wl, seed, precision, steps, warm, torch)
            tried[key] = t if bool(torch.equal(f, f_base)) else float("inf")
            log(f"seed {seed}: {t:.2f} us/step")
        b, bt = descend(seed, tried[key])
        if bt < best_t:
            best, best_t = b, bt
    return dict(params=best, us_per_step=best_t, default_us_per_step=t_base,
                candidates=len(tried), when=time.strftime("%Y-%m-%d %H:%M:%S"))


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawTextHelpFormatter)
    ap.add_argument("--workload", action="append", required=True)
    ap.add_argument("--precision", default="fp32")
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warm", type=int, default=20)
    ap.add_argument("--seed", action="append", default=[], help="extra starting point (JSON)")
    ap.add_argument("--seeds-only", action="store_true",
                    help="descend only from the cached optimum and the --seed points")
    args = ap.parse_args(argv)

    import torch

    from . import workloads as W

    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    cache = {}
    if os.path.exists(CACHE):
        with open(CACHE) as f:
            cache = json.load(f)
    for name in args.workload:
        wl = W.get(name)
        print(f"tuning {wl.name} ({args.precision}) on {arch}", flush=True)
        prev = cache.get(_key(arch, name, args.precision), {}).get("params")
        seeds = ([prev] if prev else []) + [json.loads(j) for j in args.seed]
        res = tune(wl, args.precision, args.steps, args.warm,
                   log=lambda *a: print(*a, flush=True), seeds=seeds,
                   from_defaults=not args.seeds_only)
        print(json.dumps(res), flush=True)
        cache[_key(arch, name, args.precision)] = res
        with open(CACHE + ".tmp", "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
        os.replace(CACHE + ".tmp", CACHE)
    return 0


if __name__ == "__main__":
    sys.exit(main())
