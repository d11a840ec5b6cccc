"""Precision record: the error of each precision of the GPU path against the FP64 oracle.

    python tests/precision_record.py [--workloads small,moving,sweep1024,precision,large]
                                     [--out profiles/precision_errors.json] [--procs 8]

The paper states no precision (Sections IV-VI), so this record is the statement: for every
workload and every arithmetic of the library (FP32, FP32 with compensated summation in the
column loop, FP64) the library runs the workload's T steps in the benchmark's launch
configuration, with the measurement and rebalance after every window of R steps, and is
compared with the CPU oracle in FP64:
  - over the whole field for the grids the oracle finishes in seconds (64x64x32, 256x256x64,
    512x512x64; the sweep's four chunk counts share one field, since the chunk map does not
    change any value);
  - over sampled 16x16-column windows for the 1024x1024x64 and 2048x2048x80 grids, each
    advanced by the oracle from the seeded values of a window T columns wider on every
    side, which is exact in its interior.
Reported for every run (the readings of the 1e-5 relative bar):
  eps          max |gpu - ref| / max |ref| over the compared cells
  rms_rel      sqrt(mean (gpu - ref)^2) / sqrt(mean ref^2)
  beyond       cells with |gpu - ref| > 1e-5 max |ref|, up to 16 of them listed
               (x, y, z, trip count of the last step, gpu, ref)
  one_step     the error of one more step taken from the GPU's own state, against the
               oracle's FP64 step from that same state (the FP32 parity bar)
The oracle references are computed first, in worker processes, before this process touches
the GPU.  Test infrastructure: it imports the oracle.
"""
from __future__ import annotations

import argparse
import json
import multiprocessing as mp
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from paper_1310_4218_amd import workloads as W  # noqa: E402

TOL = 1e-5
WINDOWED = {"precision", "large"}
WIN = 16


def windows(wl, T):
    """Origins of the sampled windows: the hotspot at the first and at the last step, a
    window across the periodic corner and one at an arbitrary place."""
    out = []
    for t in (0, T - 1):
        hx, hy, vx, vy = wl.hot[0]
        out.append(((hx + vx * (wl.t0 + t) - WIN // 2) % wl.nx, (hy + vy * (wl.t0 + t) - WIN // 2) % wl.ny))
    out.append((wl.nx - WIN // 2, wl.ny - WIN // 2))
    out.append((wl.nx // 3, 7))
    seen, uniq = set(), []
    for o in out:
        if o not in seen:
            seen.add(o)
            uniq.append(o)
    return uniq


def _oracle_window(args):
    """The oracle's window, advanced ten steps per call (continuing a window from its own
    output at the next time index is the same computation), with a line per piece."""
    name, ox, oy, T = args
    wl = W.get(name)
    q = oracle.init_window(wl, ox - T, oy - T, WIN + 2 * T, WIN + 2 * T)
    done = 0
    while done < T:
        n = min(10, T - done)
        q = oracle.run_window(wl, q, ox - T, oy - T, n, t0=wl.t0 + done)
        done += n
        print(f"  oracle {name} window ({ox},{oy}): {done}/{T} steps", flush=True)
    return (ox, oy), q[T:T + WIN, T:T + WIN]


def _oracle_whole(name):
    wl = W.get(name)
    q, _, _, _ = oracle.run(wl)
    return q


def gpu_run(name, precision, T):
    """The workload's T steps in the benchmark's launch configuration; returns the grid."""
    from paper_1310_4218_amd.autotune import tuned_params
    from paper_1310_4218_amd.grid import Grid
    from paper_1310_4218_amd import _abi

    wl = W.get(name)
    p = tuned_params(name, precision)
    try:
        cfg, _keep = _abi.config_from_workload(wl, precision=precision, **p)
        _abi.query(cfg)
    except _abi.LbError:          # a tile shape tuned for FP32 that FP64 rows cannot take
        p = {k: v for k, v in p.items() if k not in ("tile_x", "tile_y")}
    R = wl.rebalance_every or T
    g = Grid(wl, precision=precision, graph_steps=min(R, T), **p)
    done = 0
    while done < T:
        n = min(R, T - done)
        g.step(n, "persistent_eager")
        done += n
        g.measure("work")
        if done < T and wl.rebalance_every:
            g.rebalance(wl.strategy, wl.threshold)
    return g, p


def errors(got, ref, kfield=None, origin=(0, 0)):
    d = np.abs(got - ref)
    scale = float(np.abs(ref).max())
    eps = float(d.max() / scale)
    rms = float(np.sqrt(np.mean((got - ref) ** 2)) / np.sqrt(np.mean(ref ** 2)))
    bad = np.argwhere(d > TOL * scale)
    listed = []
    for y, x, z in bad[:16]:
        gx, gy = origin[0] + int(x), origin[1] + int(y)
        listed.append(dict(x=gx, y=gy, z=int(z), k=None if kfield is None else int(kfield[gy % kfield.shape[0], gx % kfield.shape[1]]),
                           gpu=float(got[y, x, z]), ref=float(ref[y, x, z])))
    return dict(eps=eps, rms_rel=rms, beyond=int(len(bad)), beyond_cells=listed, scale=scale)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawTextHelpFormatter)
    ap.add_argument("--workloads", default="small,moving,sweep1024,precision,large")
    ap.add_argument("--precisions", default="fp32,fp32_kahan,fp64")
    ap.add_argument("--out", default=os.path.join(ROOT, "profiles", "precision_errors.json"))
    ap.add_argument("--procs", type=int, default=8)
    args = ap.parse_args(argv)
    names = args.workloads.split(",")
    precs = args.precisions.split(",")

    # 1. oracle references (CPU, worker processes, before any GPU work)
    t = time.time()
    refs = {}
    jobs = [(n, ox, oy, W.get(n).steps) for n in names if n in WINDOWED for ox, oy in windows(W.get(n), W.get(n).steps)]
    whole = [n for n in names if n not in WINDOWED]
    with mp.get_context("fork").Pool(args.procs) as pool:
        wres = pool.map_async(_oracle_window, jobs)
        hres = pool.map_async(_oracle_whole, whole)
        for (n, ox, oy, T), (o, ref) in zip(jobs, wres.get()):
            refs.setdefault(n, {})[o] = ref
        for n, q in zip(whole, hres.get()):
            refs[n] = q
    print(f"oracle references: {time.time() - t:.1f} s", flush=True)

    # 2. GPU runs
    import torch

    if not torch.cuda.is_available():
        raise SystemExit("precision_record needs a GPU")
    record = dict(tolerance=TOL, window=WIN, workloads={})
    for n in names:
        wl = W.get(n)
        T = wl.steps
        kl = oracle.kfield(wl.nx, wl.ny, wl.hot, wl.t0 + T - 1, wl.sigma, wl.kmin, wl.kmax)
        rec = dict(grid=[wl.nx, wl.ny, wl.nz], steps=T, compared="windows" if n in WINDOWED else "whole field",
                   precisions={})
        for prec in precs:
            t = time.time()
            g, launch = gpu_run(n, prec, T)
            if n in WINDOWED:
                q = g.field(device="cuda")
                per = []
                got_all, ref_all = [], []
                for (ox, oy), ref in refs[n].items():
                    ys = torch.arange(oy, oy + WIN, device=q.device) % wl.ny
                    xs = torch.arange(ox, ox + WIN, device=q.device) % wl.nx
                    got = q[ys][:, xs].double().cpu().numpy()
                    e = errors(got, ref, kl, (ox, oy))
                    e["origin"] = [ox, oy]
                    per.append(e)
                    got_all.append(got)
                    ref_all.append(ref)
                tot = errors(np.concatenate(got_all, axis=0), np.concatenate(ref_all, axis=0))
                tot.pop("beyond_cells")
                tot["windows"] = per
                # one more step from the GPU's own state, on 18x18 windows around the same origins
                before = g.field(device="cuda")
                g.step(1, "persistent_eager")
                after = g.field(device="cuda")
                scale = float(after.abs().max())
                worst = 0.0
                for (ox, oy) in refs[n]:
                    ys = torch.arange(oy - 1, oy + WIN + 1, device=q.device) % wl.ny
                    xs = torch.arange(ox - 1, ox + WIN + 1, device=q.device) % wl.nx
                    q0 = before[ys][:, xs].double().cpu().numpy()
                    r1 = oracle.run_window(wl, q0, ox - 1, oy - 1, 1, t0=wl.t0 + T)[1:1 + WIN, 1:1 + WIN]
                    ys = torch.arange(oy, oy + WIN, device=q.device) % wl.ny
                    xs = torch.arange(ox, ox + WIN, device=q.device) % wl.nx
                    worst = max(worst, float(np.abs(after[ys][:, xs].double().cpu().numpy() - r1).max()) / scale)
                tot["one_step"] = worst
            else:
                got = np.stack([g.field(f).numpy().astype(np.float64) for f in range(wl.nfields)])
                tot = errors(got[0], refs[n][0], kl)
                before = got
                g.step(1, "persistent_eager")
                after = np.stack([g.field(f).numpy().astype(np.float64) for f in range(wl.nfields)])
                r1, _, _, _ = oracle.run(wl.replace(t0=wl.t0 + T), q0=before, nsteps=1)
                tot["one_step"] = float(np.abs(after - r1).max() / np.abs(r1).max())
            tot["launch"] = launch
            tot["seconds"] = round(time.time() - t, 1)
            g.close()
            rec["precisions"][prec] = tot
            print(n, prec, json.dumps({k: v for k, v in tot.items() if k not in ("windows", "beyond_cells")}),
                  flush=True)
        record["workloads"][n] = rec
    with open(args.out, "w") as f:
        json.dump(record, f, indent=1)
    print("wrote", args.out, flush=True)


if __name__ == "__main__":
    main()
