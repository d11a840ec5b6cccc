"""Benchmark: grid point-updates/s and max/avg slot-load ratio, balanced vs plain, 1 GPU.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload large]

A step is one time step of the whole hot path on the synthetic workload: the
cost field, the 7-point update, the column physics, the per-chunk load
measurement and the FP64 checksum, all in the library's HIP kernels; every
R steps (R = 10 for every workload) the loads of the window are read back and
the workload's balancer (GreedyLB, RefineLB or Greedy then RefineSwap) remaps
the chunks onto the slots (the paper's migration point, Section VI), which also
rebuilds the cost-ordered work items.  Two paths are timed on the same inputs:
  balanced: one launch per step over all chunks (launched step by step) in the
            workload's tuned form (one workgroup per item, or persistent
            workgroups on per-slot queues), measurement + rebalance every R
            steps, all inside the timed region; the host remaps while the
            first steps of the next window run (--overlap-steps);
  plain:    one launch per chunk over its tiles, in chunk-id order, no
            balancing (the static decomposition); timed twice, with the
            launches enqueued one by one and replayed from a captured graph.
``value`` is the balanced path's point-updates/s (cells x steps / wall time),
of the median of --repeats timed runs on fresh contexts.
The default workload is the largest single-GPU configuration: the 2048x2048x80
grid in 4096 uneven (Dirichlet) chunks with a hotspot moving diagonally two
cells per step (k in 1..400, sigma 64), RefineLB (threshold 1.05) onto 256
slots every 10 steps.

A third, ablation leg isolates the balancer (the paper's before/after
comparison of Section VI, Tables III-V): the persistent kernel with one
queue per slot and no stealing, so that the chunk->slot map alone decides
which workgroups run which chunk, with the static block map, with the
workload's balancer and with GreedyLB, each re-costed from its measured loads
every window.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_1310_4218_amd.traffic import kernel_source_hash  # noqa: E402

HBM_PEAK_GBS = 8000.0
# Vector ALU peaks of the MI355X: 256 CUs x 64 lanes x 2 flops (FMA) x 2.4 GHz = 78.6
# TFLOP/s in FP32 and in FP64.  The FP32 figure of 157.3 needs packed FP32 (two FMAs per
# lane and instruction), which this build disables (-packed-fp32-ops off).
FP32_VECTOR_PEAK_TFLOPS = 78.6
FP64_VECTOR_PEAK_TFLOPS = 78.6
METRIC = "grid point-updates/s and max/avg chunk-load ratio, balanced vs plain, 1 MI355X"
# Steps of a window are launched one by one (LB_PERSISTENT_EAGER): after each
# rebalance the first step then starts as soon as its launch is queued, where
# a graph replay first submits all R launches; measured on the default
# workload this saves about 1 us per step (the kernels are identical).
MODE = "persistent_eager"


def measured_traffic(workload: str, precision: str, launch: dict):
    """HBM bytes per launch of the persistent kernel from the committed rocprofv3
    counter summary, if it was taken on the current kernel source, in this
    precision and with this launch shape; else None."""
    name = workload if precision == "fp32" else f"{workload}_{precision}"
    path = os.path.join(ROOT, "profiles", f"traffic_{name}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if (t.get("kernel_source_hash") != kernel_source_hash() or t.get("precision", "fp32") != precision
            or t.get("launch") != launch):
        return None
    return t.get("hbm_bytes_per_launch")


def measured_valu(workload: str, precision: str, launch: dict):
    """Vector instructions per launch of the step kernel from the committed
    rocprofv3 counter record (SQ_INSTS_VALU), if it was taken on the current
    kernel source, in this precision and with this launch shape; else None."""
    name = workload if precision == "fp32" else f"{workload}_{precision}"
    path = os.path.join(ROOT, "profiles", f"counters_{name}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if (t.get("kernel_source_hash") != kernel_source_hash() or t.get("precision", "fp32") != precision
            or t.get("launch") != launch):
        return None
    return t.get("means_per_dispatch", {}).get("SQ_INSTS_VALU")


# Vector issue of the chip: 256 CUs x 4 SIMDs, each 16 lanes wide, so a wave's
# vector instruction holds its SIMD for 4 cycles; 2.4 GHz.
SIMDS = 1024
CYCLES_PER_WAVE_INSTRUCTION = 4
CLOCK_HZ = 2.4e9


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def run_balanced(Grid, wl, steps, warmup, R, params, torch, overlap=2):
    """The balanced path: windows of R steps; after each window except the last
    (the rebalance points R, 2R, ... before the end) the window's loads are
    snapshotted, the next window's first `overlap` steps are enqueued, and only
    then does the host wait for the snapshot and remap, so that the balancer and
    the plan build run while those steps run on the GPU; the new plan serves the
    window's other steps.  The warm-up ends with a rebalance, so the timed steps
    start from a measured plan.  Every kernel launch is timed with HIP events on
    the library's stream (the snapshot and plan-upload kernels between them are
    not)."""
    g = Grid(wl, graph_steps=R, **params)
    stream = g.stream
    evs = []

    def timed_steps(n, timed):
        if n <= 0:
            return
        if timed:
            e = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
            e[0].record(stream)
        g.step(n, MODE)
        if timed:
            e[1].record(stream)
            evs.append(e + (n,))

    def run(nsteps, timed):
        wins = []
        done = min(R, nsteps)
        timed_steps(done, timed)
        while done < nsteps:
            n = min(R, nsteps - done)
            g.measure_begin("work")          # the window's loads: the paper's measurement point
            timed_steps(min(overlap, n), timed)   # next window's first steps, on the plan in force
            loads = g.measure_end()          # waits for the snapshot only
            m, nmig, lam = g.rebalance(wl.strategy, wl.threshold)
            wins.append((loads, nmig, lam))
            timed_steps(n - min(overlap, n), timed)
            done += n
        return wins

    # the first step runs the unmeasured initial plan; remap after it so that the rest
    # of the warm-up (and a profile of the whole run) runs measured plans
    if warmup > 1:
        g.step(1, MODE)
        g.measure("work")
        g.rebalance(wl.strategy, wl.threshold)
    run(warmup - 1 if warmup > 1 else warmup, False)
    if warmup > 0:
        g.measure("work")
        g.rebalance(wl.strategy, wl.threshold)
    g.measure("work")                        # fresh window and busy counters
    st0 = g.stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    wins = run(steps, True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kernel_s = sum(e[0].elapsed_time(e[1]) for e in evs) / 1e3
    # launches of the step kernel in the timed region: two steps per launch when fused,
    # an odd count ending on a single step
    fused = params.get("fuse_steps") == 2
    launches = sum(n // 2 + n % 2 if fused else n for _, _, n in evs)
    # workgroup busy time of the persistent kernel over one more window
    g.step(R, MODE)
    busy = g.wg_busy()
    g.measure("work")
    st = g.stats()
    g.close()
    nw = max(len(wins), 1)
    host = dict(balance_us_per_window=(st["host_balance_us"] - st0["host_balance_us"]) / nw,
                plan_us_per_window=(st["host_plan_us"] - st0["host_plan_us"]) / nw)
    return dict(wall=wall, kernel_s=kernel_s, launches=launches, wins=wins, busy=busy, stats=st, host=host)


def run_plain(Grid, wl, steps, warmup, params, torch, mode="plain"):
    """The paper's static form: one launch per chunk and step (mode "plain"), or
    the same launches replayed from a captured graph ("plain_graph"), which
    separates the cost of launching from the cost of imbalance."""
    p = {k: v for k, v in params.items() if k in ("tile_x", "tile_y")}
    g = Grid(wl, **p)
    g.step(warmup, mode)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.step(steps, mode)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    g.close()
    return dict(wall=wall, steps=steps)


def host_description() -> dict:
    """nproc, the CPUs this process may run on and the CPU model of the host."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return dict(nproc=os.cpu_count(), affinity_cpus=len(os.sched_getaffinity(0)), cpu_model=model)


def cpu_baseline(wl, budget_s):
    """The single-threaded FP64 C oracle on the same workload, pinned in-process to one
    core (the lowest CPU this process may use): steps from the seeded field, as many as
    fit in about budget_s seconds (at least one).  The timed calls include one copy of
    the input field per call."""
    import oracle

    host = host_description()
    allowed = os.sched_getaffinity(0)
    cpu = min(allowed)
    os.sched_setaffinity(0, {cpu})
    try:
        q0 = oracle.init_field(wl.nx, wl.ny, wl.nz, wl.seed, wl.nfields)
        t = time.perf_counter()
        oracle.run(wl, q0=q0, nsteps=1)
        one = max(time.perf_counter() - t, 1e-6)
        n = max(1, min(wl.steps, int(budget_s / one)))
        if n == 1:
            dt = one
        else:
            t = time.perf_counter()
            oracle.run(wl, q0=q0, nsteps=n)
            dt = time.perf_counter() - t
    finally:
        os.sched_setaffinity(0, allowed)
    return dict(value=wl.ncells * wl.nfields * n / dt, unit="point-updates/s", cores=1,
                kind="oracle", pinned_cpu=cpu, **host,
                sample=f"{n} step(s) of the {wl.name} workload from its seeded field "
                       "(single-threaded FP64 C oracle, pinned to one core)")


def run_ablation(Grid, wl, steps, warmup, R, params, torch, balance_host):
    """The balancer's own effect: one queue per slot, no stealing, the persistent kernel
    with the same items, the static block map against the balancer's map (and against
    GreedyLB at every rebalance point when the workload's strategy is another one).
    Every window each leg measures its loads and re-installs its map with those costs
    (lb_set_map), the balanced legs after remapping from the map in force."""
    import numpy as np

    S = wl.nslots
    p = {k: v for k, v in params.items() if k not in ("nqueues", "steal", "wg_per_queue", "item_grid", "fuse_steps",
                                                         "lane_levels", "xcd_group")}
    block = np.array([(c * S) // wl.nchunks if wl.nchunks >= S else c for c in range(wl.nchunks)],
                     dtype=np.int32)
    out = {}
    legs = ("block", "balanced") + (("greedy",) if wl.strategy != "greedy" else ())
    for leg in legs:
        g = Grid(wl, graph_steps=R, nqueues=S, steal=0, wg_per_queue=0, **p)
        m = block.copy()
        first = True
        lam_in_force, lam_star, us = [], [], []
        done = -warmup
        while done < steps:
            n = R
            timed = done >= 0
            if timed:
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(g.stream)
            g.step(n, MODE)
            if timed:
                e1.record(g.stream)
            w = g.measure("work")
            if timed:
                torch.cuda.synchronize()
                us.append(e0.elapsed_time(e1) * 1e3 / n)
                L = np.bincount(m, weights=w, minlength=S)
                lam_in_force.append(float(L.max() / (w.sum() / S)))
                lam_star.append(float(max(1.0, S * w.max() / w.sum())))
            if leg != "block":
                strat = wl.strategy if leg == "balanced" else "greedy"
                if strat == "greedy_then_refineswap":
                    strat = "greedy" if first else "refineswap"
                m, _ = balance_host(w, S, strat, None if (first and strat == "greedy") else m,
                                    wl.threshold)
                first = False
            g.set_map(m, w)
            done += n
        st = g.stats()
        g.close()
        out[leg] = dict(us_per_step=float(np.mean(us)), lambda_map_in_force=float(np.mean(lam_in_force)),
                        lambda_star=float(np.mean(lam_star)), queues=st["nqueues"], workgroups=st["nwg"])
    out["speedup_balanced_over_block"] = out["block"]["us_per_step"] / out["balanced"]["us_per_step"]
    return out


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawTextHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="large")
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp32_kahan", "fp64"])
    ap.add_argument("--vertical", action="store_true",
                    help="column physics with the vertical dependency (Figs. 1 and 4)")
    ap.add_argument("--plain-steps", type=int, default=None)
    ap.add_argument("--cpu-budget", type=float, default=12.0, help="seconds of oracle work")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-ablation", action="store_true", help="skip the block-vs-balanced map leg")
    ap.add_argument("--ablation-steps", type=int, default=50)
    ap.add_argument("--repeats", type=int, default=5,
                    help="timed runs of the balanced path (fresh context each); the median is reported")
    ap.add_argument("--overlap-steps", type=int, default=2,
                    help="steps enqueued after each window before the host waits for its loads")
    ap.add_argument("--no-tuned", action="store_true", help="library default launch shape")
    ap.add_argument("--set", action="append", default=[], help="launch override key=value")
    ap.add_argument("--calibration-copy", type=float, default=0.0, metavar="MIB",
                    help="after the run, copy MIB MiB device to device (counter calibration)")
    args = ap.parse_args(argv)

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): this build has "
              "no multi-GPU path", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    from paper_1310_4218_amd import workloads as W
    from paper_1310_4218_amd._abi import balance_host
    from paper_1310_4218_amd.autotune import tuned_params
    from paper_1310_4218_amd.grid import Grid

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    wl = W.get(args.workload)
    if args.vertical:
        wl = wl.replace(vertical=1)
    R = wl.rebalance_every or 10
    S = wl.nslots
    params = {} if args.no_tuned else tuned_params(args.workload, args.precision,
                                                   physics="vertical" if args.vertical else "pointwise")
    for kv in args.set:
        k, v = kv.split("=")
        params[k] = int(v)
    params["precision"] = args.precision
    log(f"bench: {wl.name} steps={args.steps} warmup={args.warmup} R={R} S={S} params={params}")

    # the timed region is repeated on fresh contexts and the median run is reported
    runs = [run_balanced(Grid, wl, args.steps, args.warmup, R, params, torch, args.overlap_steps)
            for _ in range(max(1, args.repeats))]
    runs.sort(key=lambda r: r["wall"])
    bal = runs[len(runs) // 2]
    if len(runs) > 1:
        log("balanced runs, ms/step: " + " ".join(f"{r['wall'] * 1e3 / args.steps:.4f}" for r in runs))
    log(f"balanced: {bal['wall'] * 1e3 / args.steps:.4f} ms/step, "
        f"kernel {bal['kernel_s'] * 1e6 / args.steps:.2f} us/step")
    plain = plain_graph = None
    if not args.no_plain:
        ps = args.plain_steps or min(args.steps, 100)
        plain = run_plain(Grid, wl, ps, max(1, args.warmup // 4), params, torch)
        log(f"plain: {plain['wall'] * 1e3 / ps:.4f} ms/step")
        plain_graph = run_plain(Grid, wl, ps, max(1, args.warmup // 4), params, torch, "plain_graph")
        log(f"plain, graph replay: {plain_graph['wall'] * 1e3 / ps:.4f} ms/step")

    ablation = None
    if not args.no_ablation and wl.nchunks > 1:
        ablation = run_ablation(Grid, wl, args.ablation_steps, R, R, params, torch, balance_host)
        log(f"ablation (one queue per slot, no stealing): block {ablation['block']['us_per_step']:.1f} "
            f"us/step, balanced {ablation['balanced']['us_per_step']:.1f} us/step")

    cells = wl.ncells * wl.nfields
    value = cells * args.steps / bal["wall"]
    plain_value = cells * plain["steps"] / plain["wall"] if plain else None
    plain_graph_value = cells * plain_graph["steps"] / plain_graph["wall"] if plain_graph else None

    def lam_of(w, m):
        L = np.bincount(m, weights=w, minlength=S)
        return float(L.max() / (w.sum() / S))

    block = np.array([(c * S) // wl.nchunks if wl.nchunks >= S else c for c in range(wl.nchunks)])
    loads = [w for w, _, _ in bal["wins"]]
    # map in force vs its window (None when the timed steps hold no rebalance point)
    lam_bal = float(np.mean([lam[0] for _, _, lam in bal["wins"]])) if loads else None
    lam_plain = float(np.mean([lam_of(w, block) for w in loads])) if loads else None
    lam_star = float(np.mean([max(1.0, S * w.max() / w.sum()) for w in loads])) if loads else None
    # per persistent workgroup, or per compute unit that ran items (one workgroup per item)
    busy = bal["busy"]
    busy = busy[busy > 0] if params.get("item_grid") else busy
    lam_wg = float(busy.max() / busy.mean()) if busy.size and busy.mean() > 0 else None

    elem = 8 if args.precision == "fp64" else 4
    # Algorithmic bytes: 2 * elem per point-update (one read, one write), times the
    # point-updates a launch makes (cells x the steps it takes).  A launch of two steps
    # moves each cell once for both, so its compulsory traffic is half of that: the
    # per-update figure can then exceed the peak, and the compulsory fraction is given
    # beside it.
    kernel_launch_s = bal["kernel_s"] / bal["launches"]
    steps_per_launch = args.steps / bal["launches"]
    bytes_per_update = 2 * elem
    units_per_launch = cells * steps_per_launch
    compulsory_bytes = 2 * elem * cells
    # both field copies larger than the 256 MB Infinity Cache: every step streams from HBM;
    # smaller grids stay cache-resident and are bound by latency and fixed costs instead
    hbm_resident = compulsory_bytes > 256 * 2 ** 20
    achieved = bytes_per_update * units_per_launch / kernel_launch_s / 1e9
    compulsory_gbs = compulsory_bytes / kernel_launch_s / 1e9
    fused = params.get("fuse_steps") == 2
    kname = ("k_items2" if fused else "k_items") if params.get("item_grid") else "k_persistent"
    # Algorithmic floating-point operations of one step: 8 per point update for the
    # stencil and its combination (5 additions of the six neighbours, cc*c + cn*sum) and 5 per iteration of the
    # column physics (q*q*q, the difference, the scaling by eps, the sum).  The trip
    # counts summed over the grid follow from the measured work loads of the timed
    # windows (work = nz * nfields * (alpha * columns + sum of trip counts), R steps each).
    cols = wl.nx * wl.ny
    ksum_step = (float(np.mean([w.sum() for w in loads])) / (wl.nz * wl.nfields) - wl.alpha_work * cols * R) / R \
        if loads else None
    flops_step = 8.0 * cells + 5.0 * wl.nz * wl.nfields * ksum_step if ksum_step is not None else None
    flops_launch = flops_step * steps_per_launch if flops_step is not None else None
    tflops = flops_launch / kernel_launch_s / 1e12 if flops_launch is not None else None
    alu_peak = FP64_VECTOR_PEAK_TFLOPS if args.precision == "fp64" else FP32_VECTOR_PEAK_TFLOPS
    st = bal["stats"]
    alu = {"achieved": tflops, "peak": alu_peak, "unit": "TFLOP/s",
           "frac": tflops / alu_peak if tflops is not None else None, "flops_per_launch": flops_launch}
    # HBM-resident grids are reported against HBM, cache-resident ones as latency-bound;
    # the ALU view is beside it (the two-step launch also keeps the vector units busy).
    roof = {"bound": "hbm" if hbm_resident else "latency", "achieved": achieved, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
            "traffic": (measured_traffic(args.workload, args.precision,
                                         {k: v for k, v in params.items() if k != "precision"})
                        if not args.vertical else None),   # the records are of the pointwise kernel
            "kernel": kname, "bytes_per_update": bytes_per_update, "units_per_launch": units_per_launch,
            "steps_per_launch": steps_per_launch,
            "compulsory": {"bytes_per_launch": compulsory_bytes, "achieved": compulsory_gbs,
                           "frac": compulsory_gbs / HBM_PEAK_GBS},
            "alu": alu, "us_per_launch_events": kernel_launch_s * 1e6}
    # Vector issue: the counted vector instructions of a launch over the issue slots of
    # its duration (every SIMD issuing one wave instruction per 4 cycles at 2.4 GHz).
    launch_cfg = {k: v for k, v in params.items() if k != "precision"}
    valu = measured_valu(args.workload, args.precision, launch_cfg) if not args.vertical else None
    roof["issue"] = {"valu_instructions_per_launch": valu,
                     "frac": (valu * CYCLES_PER_WAVE_INSTRUCTION / (SIMDS * CLOCK_HZ * kernel_launch_s)
                              if valu else None)}

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "point-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": bal["wall"] * 1e3 / args.steps,
        "repeats": len(runs),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32": "f32", "fp32_kahan": "f32", "fp64": "f64"}[args.precision],
        "data": "synthetic",
        "config": {"workload": wl.name, "grid": [wl.nx, wl.ny, wl.nz], "chunks": wl.nchunks,
                   "physics": "vertical" if args.vertical else "pointwise",
                   "slots": S, "rebalance_every": R, "strategy": wl.strategy,
                   "overlap_steps": args.overlap_steps,
                   "launch": {k: v for k, v in params.items() if k != "precision"},
                   "workgroups": st["nwg"], "tiles": st["ntiles"], "items": st["nitems"]},
        "balanced_vs_plain": {
            "balanced_point_updates_per_s": value,
            "plain_point_updates_per_s": plain_value,
            "speedup": value / plain_value if plain_value else None,
            "plain_graph_point_updates_per_s": plain_graph_value,
            "speedup_vs_plain_graph": value / plain_graph_value if plain_graph_value else None,
            "lambda_balanced": lam_bal,
            "lambda_plain": lam_plain,
            "lambda_star": lam_star,
            "lambda_wg": lam_wg,
            "lambda_wg_over": "compute units" if params.get("item_grid") else "workgroups",
            "busy_units": int(busy.size),
            "queues": st["nqueues"],
            "map_inert": st["nqueues"] == 1,
            "migrations_per_rebalance": float(np.mean([n for _, n, _ in bal["wins"]])) if bal["wins"] else None,
            "host_us_per_window": bal["host"],
        },
        "ablation_map_only": ablation,
        "roofline": roof,
    }
    if args.calibration_copy > 0:
        n = int(args.calibration_copy * 2 ** 20)
        src = torch.ones(n, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        out["calibration_copy_bytes"] = n
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(wl, args.cpu_budget)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
