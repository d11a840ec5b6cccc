"""HBM traffic of the step kernel (k_items2, k_items or k_persistent) from two rocprofv3 counter runs.

    rocprofv3 --pmc FETCH_SIZE -d OUT/fetch -o run -- python3 bench.py --workload W \
        --no-cpu --no-plain --no-ablation --steps S --warmup 10 --calibration-copy 512
    rocprofv3 --pmc WRITE_SIZE -d OUT/write -o run -- python3 bench.py ...same...
    python -m paper_1310_4218_amd.traffic --fetch OUT/fetch --write OUT/write --workload W \
        --copy-mib 512
    python -m paper_1310_4218_amd.traffic stats OUT/stats --title T --command C --write F.md
    python -m paper_1310_4218_amd.traffic counters OUT/pmc --kernel k_items2 --title T \
        --command C --write F.md [--workload W [--precision P]]

Both counters are reported in KiB per dispatch.  Each is scaled by what the
same counter reads for the plain device copy of known size that bench.py runs
in the same process (--calibration-copy), so the result is in bytes as the
counter sees them for a kernel whose true traffic is known.  Writes
profiles/traffic_<workload>.json (traffic_<workload>_<precision>.json outside
FP32): per-launch bytes, the scale factors, the precision, the launch shape
from tuned.json and a hash of the kernel source, so that bench.py reports the
figure only for the kernel, precision and launch shape it was taken on.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import re
import sys

from .autotune import tuned_params

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def kernel_source_hash() -> str:
    """Hash of the device code's tokens (comments and layout removed), so that a
    counter record stays valid across comment-only edits and no longer after a
    code change."""
    h = hashlib.sha256()
    for f in ("kernels.hip", "lbgrid_internal.h"):
        with open(os.path.join(ROOT, "paper_1310_4218_amd", "csrc", f)) as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def read_counter(outdir: str, counter: str):
    """{kernel name: [value per dispatch]} from rocprofv3 counter CSVs under outdir."""
    per = {}
    files = glob.glob(os.path.join(outdir, "**", "*counter_collection*.csv"), recursive=True)
    if not files:
        raise FileNotFoundError(f"no counter_collection CSV under {outdir}")
    for path in files:
        with open(path, newline="") as f:
            for row in csv.DictReader(f):
                if row.get("Counter_Name") != counter:
                    continue
                name = row.get("Kernel_Name", "")
                per.setdefault(name, []).append(float(row["Counter_Value"]))
    return per


def pick(per: dict, needle) -> list:
    vals = []
    for name, v in per.items():
        if any(n in name.lower() for n in needle):
            vals.extend(v)
    return vals


def stats_summary(outdir: str, title: str, command: str, top: int = 12) -> str:
    """Markdown table of the per-kernel statistics rocprofv3 --stats wrote under outdir."""
    files = glob.glob(os.path.join(outdir, "**", "*kernel_stats.csv"), recursive=True)
    if not files:
        raise FileNotFoundError(f"no kernel_stats CSV under {outdir}")
    rows = []
    for path in files:
        with open(path, newline="") as f:
            rows.extend(csv.DictReader(f))
    rows.sort(key=lambda r: -float(r.get("TotalDurationNs", 0)))
    # per-kernel median duration from the dispatch trace, when it was written too
    durs = {}
    for path in glob.glob(os.path.join(outdir, "**", "*kernel_trace.csv"), recursive=True):
        with open(path, newline="") as f:
            for t in csv.DictReader(f):
                durs.setdefault(t["Kernel_Name"], []).append(
                    int(t["End_Timestamp"]) - int(t["Start_Timestamp"]))
    out = [f"# {title}", "", "Command:", "", "```", command, "```", "",
           "| kernel | calls | total ms | average us | median us | min us | max us | % |",
           "|---|---|---|---|---|---|---|---|"]
    for r in rows[:top]:
        name = r.get("Name", "")
        d = sorted(durs.get(name, []))
        med = "{:.2f}".format(d[len(d) // 2] / 1e3) if d else "-"
        if len(name) > 70:
            name = name[:67] + "..."
        out.append("| `{}` | {} | {:.3f} | {:.2f} | {} | {:.2f} | {:.2f} | {:.1f} |".format(
            name, r.get("Calls"), float(r.get("TotalDurationNs", 0)) / 1e6,
            float(r.get("AverageNs", 0)) / 1e3, med, float(r.get("MinNs", 0)) / 1e3,
            float(r.get("MaxNs", 0)) / 1e3, float(r.get("Percentage", 0))))
    return "\n".join(out) + "\n"


def counter_means(outdir: str, kernel: str) -> dict:
    """{counter: mean per dispatch} of `kernel` under outdir (each dispatch's value
    summed over the device)."""
    per = {}
    for path in glob.glob(os.path.join(outdir, "**", "*counter_collection*.csv"), recursive=True):
        with open(path, newline="") as f:
            for row in csv.DictReader(f):
                if kernel + "<" not in row.get("Kernel_Name", ""):
                    continue
                key = (row["Counter_Name"], row["Dispatch_Id"])
                per[key] = per.get(key, 0.0) + float(row["Counter_Value"])
    out = {}
    for c in sorted({c for c, _ in per}):
        v = [x for (n, _), x in per.items() if n == c]
        out[c] = sum(v) / len(v)
    return out


def counters_summary(outdir: str, kernel: str, title: str, command: str) -> str:
    """Markdown table of every counter rocprofv3 --pmc collected under outdir for the
    dispatches of `kernel` (each dispatch's value summed over the device, then the
    mean over dispatches), with the dispatches' median duration when a kernel trace
    was written too."""
    per = {}
    for path in glob.glob(os.path.join(outdir, "**", "*counter_collection*.csv"), recursive=True):
        with open(path, newline="") as f:
            for row in csv.DictReader(f):
                if kernel + "<" not in row.get("Kernel_Name", ""):
                    continue
                key = (row["Counter_Name"], row["Dispatch_Id"])
                per[key] = per.get(key, 0.0) + float(row["Counter_Value"])
    if not per:
        raise FileNotFoundError(f"no counter values for {kernel} under {outdir}")
    names = sorted({c for c, _ in per})
    durs = []
    for path in glob.glob(os.path.join(outdir, "**", "*kernel_trace.csv"), recursive=True):
        with open(path, newline="") as f:
            for t in csv.DictReader(f):
                if kernel + "<" in t["Kernel_Name"]:
                    durs.append(int(t["End_Timestamp"]) - int(t["Start_Timestamp"]))
    out = [f"# {title}", "", "Command:", "", "```", command, "```", "",
           "| counter | dispatches | mean per dispatch |", "|---|---|---|"]
    for c in names:
        v = [x for (n, _), x in per.items() if n == c]
        out.append(f"| `{c}` | {len(v)} | {sum(v) / len(v):.4g} |")
    if durs:
        durs.sort()
        out += ["", f"Median dispatch duration under the counters: {durs[len(durs) // 2] / 1e3:.1f} us "
                    f"({len(durs)} dispatches)."]
    return "\n".join(out) + "\n"


def main(argv=None) -> int:
    if argv is None:
        argv = sys.argv[1:]
    if argv and argv[0] == "counters":
        ap = argparse.ArgumentParser(prog="traffic counters")
        ap.add_argument("outdir")
        ap.add_argument("--kernel", required=True)
        ap.add_argument("--title", required=True)
        ap.add_argument("--command", required=True)
        ap.add_argument("--write", help="markdown file to write")
        ap.add_argument("--workload", help="with --precision: also write profiles/counters_<workload>.json "
                                           "(the means, the launch shape and the kernel source hash)")
        ap.add_argument("--precision", default="fp32")
        a = ap.parse_args(argv[1:])
        md = counters_summary(a.outdir, a.kernel, a.title, a.command)
        if a.write:
            with open(a.write, "w") as f:
                f.write(md)
        if a.workload:
            name = a.workload if a.precision == "fp32" else f"{a.workload}_{a.precision}"
            rec = dict(workload=a.workload, kernel=a.kernel, precision=a.precision,
                       means_per_dispatch=counter_means(a.outdir, a.kernel),
                       launch=tuned_params(a.workload, a.precision),
                       kernel_source_hash=kernel_source_hash(), command=a.command)
            with open(os.path.join(ROOT, "profiles", f"counters_{name}.json"), "w") as f:
                json.dump(rec, f, indent=1)
        print(md)
        return 0
    if argv and argv[0] == "stats":
        ap = argparse.ArgumentParser(prog="traffic stats")
        ap.add_argument("outdir")
        ap.add_argument("--title", required=True)
        ap.add_argument("--command", required=True)
        ap.add_argument("--write", help="markdown file to write")
        a = ap.parse_args(argv[1:])
        md = stats_summary(a.outdir, a.title, a.command)
        if a.write:
            with open(a.write, "w") as f:
                f.write(md)
        print(md)
        return 0
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawTextHelpFormatter)
    ap.add_argument("--fetch", required=True)
    ap.add_argument("--write", required=True)
    ap.add_argument("--workload", required=True)
    ap.add_argument("--copy-mib", type=float, required=True)
    ap.add_argument("--precision", default="fp32")
    ap.add_argument("--command", default="", help="command lines that produced the runs")
    args = ap.parse_args(argv)

    fetch = read_counter(args.fetch, "FETCH_SIZE")
    write = read_counter(args.write, "WRITE_SIZE")
    # the step kernel: one workgroup per item, two steps or one per launch, if the run
    # launched it, else the persistent one
    kname = next((k for k in ("k_items2", "k_items", "k_persistent_march", "k_persistent")
                  if pick(fetch, [k + "<"])), "k_persistent")
    kf, kw = pick(fetch, [kname + "<"]), pick(write, [kname + "<"])
    cf, cw = pick(fetch, ["copy"]), pick(write, ["copy"])
    if not kf or not kw or not cf or not cw:
        print("missing dispatches: persistent", len(kf), len(kw), "copy", len(cf), len(cw),
              file=sys.stderr)
        print("kernels seen:", sorted(set(fetch) | set(write)), file=sys.stderr)
        return 1
    copy_bytes = args.copy_mib * 2 ** 20
    # the copy reads and writes copy_bytes; the counters report KiB per dispatch
    f_scale = copy_bytes / (max(cf) * 1024.0)
    w_scale = copy_bytes / (max(cw) * 1024.0)
    mean = lambda v: sum(v) / len(v)
    fetch_b = mean(kf) * 1024.0 * f_scale
    write_b = mean(kw) * 1024.0 * w_scale
    out = dict(workload=args.workload, kernel=kname,
               dispatches=dict(fetch=len(kf), write=len(kw)),
               fetch_bytes_per_launch=fetch_b, write_bytes_per_launch=write_b,
               hbm_bytes_per_launch=fetch_b + write_b,
               raw_kib_per_launch=dict(fetch=mean(kf), write=mean(kw)),
               calibration=dict(copy_bytes=copy_bytes, fetch_kib=max(cf), write_kib=max(cw),
                                fetch_scale=f_scale, write_scale=w_scale),
               precision=args.precision, launch=tuned_params(args.workload, args.precision),
               kernel_source_hash=kernel_source_hash(), command=args.command)
    name = args.workload if args.precision == "fp32" else f"{args.workload}_{args.precision}"
    path = os.path.join(ROOT, "profiles", f"traffic_{name}.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out, indent=1))
    return 0


if __name__ == "__main__":
    sys.exit(main())
