"""Reference bandwidths of plain streaming kernels on the current GPU.

    python -m paper_1310_4218_amd.stream_ref

Times torch's device copy, an elementwise add and a fill over 1 GiB of FP32
(HBM-resident), and the add over the 32 MiB + 32 MiB a 256^2 x 64 FP32 step
touches (MALL-resident), with HIP events over 20 (100) repetitions.  These are
the practical ceilings the step kernel's counted traffic is compared with;
nothing here belongs to the method.
"""
from __future__ import annotations

import json
import sys


def main() -> int:
    import torch

    if not torch.cuda.is_available():
        print("stream_ref needs a GPU", file=sys.stderr)
        return 1
    n = 256 * 2 ** 20                      # 1 GiB of FP32
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    out = {}

    def timed(fn, reps, nbytes):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        t = e0.elapsed_time(e1) / reps / 1e3
        return {"us": t * 1e6, "TB_per_s": nbytes / t / 1e12}

    out["copy_1GiB"] = timed(lambda: y.copy_(x), 20, 2 * 4 * n)
    out["add_1GiB"] = timed(lambda: torch.add(x, 1.0, out=y), 20, 2 * 4 * n)
    out["fill_1GiB"] = timed(lambda: y.fill_(2.0), 20, 4 * n)
    m = 2 ** 23                            # 32 MiB of FP32
    xs, ys = x[:m], y[:m]
    out["add_32MiB"] = timed(lambda: torch.add(xs, 1.0, out=ys), 100, 2 * 4 * m)
    out["device"] = torch.cuda.get_device_properties(0).gcnArchName
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
