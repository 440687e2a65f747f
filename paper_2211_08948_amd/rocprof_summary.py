"""Turns rocprofv3 CSV output into the short text summaries kept under
profiles/: a kernel-statistics table and, from two counter passes
(FETCH_SIZE, WRITE_SIZE) plus the same passes over a plain copy of known size,
the HBM bytes per launch of one kernel.

    python -m paper_2211_08948_amd.rocprof_summary stats STATS_CSV --title T --command C --out MD
    python -m paper_2211_08948_amd.rocprof_summary traffic --fetch CSV --write CSV \
        --copy-fetch CSV --copy-write CSV --copy-bytes N --kernel SUBSTR --command C --out JSON [--last N]

Counter values are KiB per dispatch.  Each is scaled by the ratio of the copy's
known bytes to what the same counter reads for the copy, so the figure is in
the copy's units (bytes that crossed the HBM interface).
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = ("csrc/kernels.hip", "csrc/device.hpp", "csrc/common.hpp")


def kernel_source_hash() -> str:
    """Hash of the sources that define the device kernels: counter figures are
    valid only for the kernel they were taken on."""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(HERE, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _rows(path):
    with open(path, newline="") as fh:
        return list(csv.DictReader(fh))


def stats_markdown(path: str, title: str, command: str, top: int = 12) -> str:
    rows = _rows(path)
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    out = [f"# {title}", "", "Command:", "", "    " + command, "",
           "| kernel | calls | total ns | avg ns | min ns | max ns | % |", "|---|---|---|---|---|---|---|"]
    for r in rows[:top]:
        name = r["Name"]
        if len(name) > 90:
            name = name[:87] + "..."
        out.append(f"| {name} | {r['Calls']} | {r['TotalDurationNs']} | {float(r['AverageNs']):.0f} | "
                   f"{r.get('MinNs', '')} | {r.get('MaxNs', '')} | {r['Percentage']} |")
    return "\n".join(out) + "\n"


def _counter_avg(path: str, counter: str, kernel_substr: str, last: int = 0):
    """Mean over the matching dispatches of one counter (KiB per dispatch);
    with last > 0 only over the last `last` of them (the timed launches, not
    the autotuner's trial launches before them)."""
    per_dispatch = {}
    for r in _rows(path):
        if r.get("Counter_Name") != counter or kernel_substr not in r.get("Kernel_Name", ""):
            continue
        key = r.get("Dispatch_Id") or r.get("Correlation_Id")
        per_dispatch[key] = per_dispatch.get(key, 0.0) + float(r["Counter_Value"])
    if not per_dispatch:
        raise SystemExit(f"no {counter} rows for kernels matching {kernel_substr!r} in {path}")
    keys = sorted(per_dispatch, key=lambda k: int(k))
    if last > 0:
        keys = keys[-last:]
    vals = [per_dispatch[k] for k in keys]
    return sum(vals) / len(vals), len(vals)


def traffic(args) -> dict:
    f_kib, nf = _counter_avg(args.fetch, "FETCH_SIZE", args.kernel, args.last)
    w_kib, nw = _counter_avg(args.write, "WRITE_SIZE", args.kernel, args.last)
    cf_kib, _ = _counter_avg(args.copy_fetch, "FETCH_SIZE", args.copy_kernel)
    cw_kib, _ = _counter_avg(args.copy_write, "WRITE_SIZE", args.copy_kernel)
    fetch_scale = args.copy_bytes / (cf_kib * 1024.0)
    write_scale = args.copy_bytes / (cw_kib * 1024.0)
    fetch_b = f_kib * 1024.0 * fetch_scale
    write_b = w_kib * 1024.0 * write_scale
    return {
        "kernel": args.kernel, "kernel_hash": kernel_source_hash(), "command": args.command,
        "dispatches": {"fetch": nf, "write": nw},
        "fetch_kib_per_dispatch": round(f_kib, 1), "write_kib_per_dispatch": round(w_kib, 1),
        "copy_bytes_each_way": args.copy_bytes,
        "copy_fetch_kib": round(cf_kib, 1), "copy_write_kib": round(cw_kib, 1),
        "fetch_scale": round(fetch_scale, 4), "write_scale": round(write_scale, 4),
        "hbm_bytes_per_launch": round(fetch_b + write_b),
        "hbm_fetch_bytes_per_launch": round(fetch_b), "hbm_write_bytes_per_launch": round(write_b),
    }


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("csv")
    s.add_argument("--title", required=True)
    s.add_argument("--command", required=True)
    s.add_argument("--out", required=True)
    t = sub.add_parser("traffic")
    for k in ("fetch", "write", "copy-fetch", "copy-write", "kernel", "command", "out"):
        t.add_argument("--" + k, required=True)
    t.add_argument("--copy-kernel", default="copy")
    t.add_argument("--copy-bytes", type=float, required=True)
    t.add_argument("--last", type=int, default=0, help="use only the last N matching dispatches")
    args = ap.parse_args(argv)
    if args.cmd == "stats":
        text = stats_markdown(args.csv, args.title, args.command)
    else:
        text = json.dumps(traffic(args), indent=1) + "\n"
    with open(args.out, "w") as fh:
        fh.write(text)
    sys.stdout.write(text)


if __name__ == "__main__":
    main()
