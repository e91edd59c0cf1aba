"""Summaries of rocprofv3 CSV output for the PCDN kernels.

    python -m paper_1306_4080_amd.profsum stats DIR --title T --cmd C > summary.md
        kernel statistics and per-launch-shape durations of a
        `rocprofv3 --kernel-trace --stats --output-format csv -d DIR -o run` run.

    python -m paper_1306_4080_amd.profsum traffic --kernel REGEX --cls NAME \
        --fetch DIR --write DIR --copy-fetch DIR --copy-write DIR --copy-bytes B \
        --source-hash H --cmd C --out profiles/NAME_c2_traffic.json
        HBM bytes per launch of the kernels matching REGEX from two counter runs
        (`--pmc FETCH_SIZE`, then `--pmc WRITE_SIZE`), each scaled by what the
        same counter reads for a plain copy kernel that reads and writes B bytes.

Only reads CSV files; nothing here touches the GPU.
"""
from __future__ import annotations

import argparse
import collections
import csv
import glob
import json
import os
import re
import sys


def _one(directory: str, suffix: str) -> str:
    hits = sorted(glob.glob(os.path.join(directory, "**", "*" + suffix), recursive=True))
    if not hits:
        raise SystemExit(f"no *{suffix} under {directory}")
    return hits[0]


def _short(name: str) -> str:
    m = re.search(r"(k_\w+)(<[^>]*>)?", name)
    return (m.group(1) + (m.group(2) or "")) if m else name[:48]


def stats(args) -> None:
    rows = list(csv.DictReader(open(_one(args.dir, "kernel_stats.csv"))))
    out = [f"# {args.title}", "", "Command (from the repository root on the GPU box):", "",
           "```", args.cmd, "```", "", "rocprofv3 kernel statistics (all dispatches of the run):",
           "", "| kernel | calls | avg us | min us | max us | total ms | % |",
           "|---|---|---|---|---|---|---|"]
    for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"])):
        if float(r["Percentage"]) < 0.05:
            continue
        out.append(f"| `{_short(r['Name'])}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
                   f"{float(r['MinNs']) / 1e3:.2f} | {float(r['MaxNs']) / 1e3:.2f} | "
                   f"{float(r['TotalDurationNs']) / 1e6:.2f} | {float(r['Percentage']):.1f} |")
    trace = list(csv.DictReader(open(_one(args.dir, "kernel_trace.csv"))))
    by = collections.defaultdict(list)
    for r in trace:
        if not re.search(r"k_\w+", r["Kernel_Name"]):
            continue
        gx = int(r["Grid_Size_X"]) // max(1, int(r["Workgroup_Size_X"]))
        gy = int(r["Grid_Size_Y"]) // max(1, int(r["Workgroup_Size_Y"]))
        by[(_short(r["Kernel_Name"]), gx, gy)].append(
            (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    out += ["", "Per launch shape (grid blocks x, y) from the kernel trace:", "",
            "| kernel | grid | launches | median us | p90 us |", "|---|---|---|---|---|"]
    for k in sorted(by, key=lambda k: -sum(by[k]))[:24]:
        v = sorted(by[k])
        out.append(f"| `{k[0]}` | {k[1]}x{k[2]} | {len(v)} | {v[len(v) // 2]:.2f} | "
                   f"{v[int(len(v) * 0.9)]:.2f} |")
    print("\n".join(out))


def _per_dispatch(directory: str, counter: str, pattern: str) -> list[float]:
    """Counter value (summed over instances) of every dispatch whose kernel
    name matches `pattern`."""
    rows = csv.DictReader(open(_one(directory, "counter_collection.csv")))
    acc = collections.OrderedDict()
    rx = re.compile(pattern)
    for r in rows:
        if r["Counter_Name"] != counter or not rx.search(r["Kernel_Name"]):
            continue
        acc[r["Dispatch_Id"]] = acc.get(r["Dispatch_Id"], 0.0) + float(r["Counter_Value"])
    if not acc:
        raise SystemExit(f"no {counter} rows for /{pattern}/ under {directory}")
    return list(acc.values())


def traffic(args) -> None:
    mean = lambda v: sum(v) / len(v)
    kf = _per_dispatch(args.fetch, "FETCH_SIZE", args.kernel)
    kw = _per_dispatch(args.write, "WRITE_SIZE", args.kernel)
    # the largest copy dispatch is the calibration copy itself
    cf = max(_per_dispatch(args.copy_fetch, "FETCH_SIZE", args.copy_kernel))
    cw = max(_per_dispatch(args.copy_write, "WRITE_SIZE", args.copy_kernel))
    f_scale = args.copy_bytes / cf      # bytes per counter unit, reads
    w_scale = args.copy_bytes / cw      # bytes per counter unit, writes
    rec = {
        "kernel_class": args.cls,
        "kernel_regex": args.kernel,
        "kernel_source_sha256_16": args.source_hash,
        "launches": {"fetch_run": len(kf), "write_run": len(kw)},
        "fetch_counter_per_launch": mean(kf),
        "write_counter_per_launch": mean(kw),
        "copy_calibration": {"bytes_read": args.copy_bytes, "bytes_written": args.copy_bytes,
                             "fetch_counter": cf, "write_counter": cw,
                             "bytes_per_fetch_unit": f_scale, "bytes_per_write_unit": w_scale},
        "hbm_read_bytes_per_launch": mean(kf) * f_scale,
        "hbm_write_bytes_per_launch": mean(kw) * w_scale,
        "hbm_bytes_per_launch": mean(kf) * f_scale + mean(kw) * w_scale,
        "command": args.cmd,
    }
    with open(args.out, "w") as f:
        json.dump(rec, f, indent=1)
        f.write("\n")
    print(json.dumps(rec, indent=1))


def main(argv=None) -> None:
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    sub = ap.add_subparsers(dest="cmd_name", required=True)
    s = sub.add_parser("stats")
    s.add_argument("dir")
    s.add_argument("--title", required=True)
    s.add_argument("--cmd", required=True)
    t = sub.add_parser("traffic")
    t.add_argument("--kernel", required=True)
    t.add_argument("--cls", required=True)
    t.add_argument("--fetch", required=True)
    t.add_argument("--write", required=True)
    t.add_argument("--copy-fetch", required=True)
    t.add_argument("--copy-write", required=True)
    t.add_argument("--copy-kernel", default=r"copy|Copy")
    t.add_argument("--copy-bytes", type=float, required=True)
    t.add_argument("--source-hash", required=True)
    t.add_argument("--cmd", required=True)
    t.add_argument("--out", required=True)
    a = ap.parse_args(argv)
    (stats if a.cmd_name == "stats" else traffic)(a)


if __name__ == "__main__":
    main(sys.argv[1:])
