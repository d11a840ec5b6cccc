"""Per-workgroup timeline of one persistent step.

    python -m paper_1310_4218_amd.timeline [--workload moving] [--reps 3]

Runs the workload's tuned launch for a few windows of R steps (each followed
by a measurement and a rebalance, as the benchmark runs), then single steps,
and after each reads the in-kernel wall-clock stamps of every workgroup
(lb_wg_timeline: start, first item, end of last item, exit).  It prints when
workgroups start, when their first item starts, and how their exits spread.
It also compares the workgroups that run one host-assigned item with those
that run two.
"""
from __future__ import annotations

import argparse
import json
import sys


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawTextHelpFormatter)
    ap.add_argument("--workload", default="moving")
    ap.add_argument("--precision", default="fp32")
    ap.add_argument("--reps", type=int, default=3)
    args = ap.parse_args(argv)

    import numpy as np
    import torch

    from . import workloads as W
    from .autotune import tuned_params
    from .grid import Grid

    wl = W.get(args.workload)
    R = wl.rebalance_every or 10
    g = Grid(wl, precision=args.precision, graph_steps=R, **tuned_params(args.workload, args.precision))
    for _ in range(4):
        g.step(R, "persistent_eager")
        g.measure("work")
        g.rebalance(wl.strategy, wl.threshold)
    torch.cuda.synchronize()
    st = g.stats()
    nwg, nit = st["nwg"], st["nitems"]
    # workgroup ranks below 2*nwg - nitems have no second host-assigned item (one queue)
    single = np.arange(nwg) < max(0, 2 * nwg - nit) if st["nqueues"] == 1 else np.zeros(nwg, bool)
    out = []
    for _ in range(args.reps):
        g.step(1, "persistent_eager")
        torch.cuda.synchronize()
        tl = g.wg_timeline()
        start, first, last, exit_ = tl[:, 0], tl[:, 1], tl[:, 2], tl[:, 3]
        rec = {
            "span_us": float(exit_.max() - start.min()),
            "start_spread_us": float(start.max() - start.min()),
            "first_item_after_start_us": {"median": float(np.median(first - start)),
                                          "max": float(np.max(first - start))},
            "exit_percentiles_us": dict(zip(("p10", "p50", "p90", "max"),
                                            map(float, np.percentile(exit_, [10, 50, 90, 100])))),
        }
        if single.any() and (~single).any():
            rec["one_item_wgs"] = {"n": int(single.sum()), "exit_mean_us": float(exit_[single].mean())}
            rec["two_item_wgs"] = {"n": int((~single).sum()), "exit_mean_us": float(exit_[~single].mean()),
                                   "exit_max_us": float(exit_[~single].max())}
        out.append(rec)
        print(json.dumps(rec), flush=True)
    g.close()
    print(json.dumps({"workload": wl.name, "workgroups": nwg, "items": nit}), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
