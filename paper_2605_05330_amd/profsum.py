"""Summaries of rocprofv3 CSV output for the step kernel's measurements.

    python -m paper_2605_05330_amd.profsum trace DIR [--last N --grid G --kernel K]
    python -m paper_2605_05330_amd.profsum traffic FETCH_DIR WRITE_DIR [--grid G --last N]
    python -m paper_2605_05330_amd.profsum counters DIR [DIR ...] [--kernel K --grid G --last N]

`trace` reads `*kernel_trace.csv` and prints, per (kernel, grid size), the call
count and the average / median / minimum duration; with --grid it also prints
the average over the last N dispatches of that kernel at that grid size (bench.py
times the step kernel over its last 1000 launches on the benchmark graph).

`traffic` reads the `*counter_collection.csv` of one FETCH_SIZE run and one
WRITE_SIZE run.  It scales each counter by what the same counter reads for the
largest plain copy (`__amd_rocclr_copyBuffer`, 64 MiB read and 64 MiB written:
bench.py issues one), and prints the HBM bytes per dispatch of the step kernel's
last N dispatches (at grid size G when it ran at several), with a JSON line that bench.py reads back.  The
line carries a hash of the step kernel's sources, so that a later change of the
kernel makes those figures stale (bench.py then reports no traffic).
"""
from __future__ import annotations

import argparse
import collections
import csv
import glob
import hashlib
import json
import os
import statistics

COPY_KERNEL = "__amd_rocclr_copyBuffer"
COPY_BYTES = 64 * 1024 * 1024
STEP_KERNEL = "wrgn_step_kernel"
_CSRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")
STEP_SOURCES = ("gn_step.hip", "gn_rowsum.h", "gn_ctl.h", "gn_types.h")


def kernel_source_hash() -> str:
    """sha256 over the step kernel's source files (first 16 hex digits)."""
    h = hashlib.sha256()
    for name in STEP_SOURCES:
        with open(os.path.join(_CSRC, name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read() + b"\0")
    return h.hexdigest()[:16]


def _rows(d: str, suffix: str):
    paths = sorted(glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True))
    if not paths:
        raise SystemExit("no *%s under %s" % (suffix, d))
    rows = []
    for p in paths:
        with open(p, newline="") as f:
            rows.extend(csv.DictReader(f))
    key = "Dispatch_Id" if "Dispatch_Id" in rows[0] else "Correlation_Id"
    rows.sort(key=lambda r: int(r[key]))
    return rows


def _grid(r) -> str:
    return r.get("Grid_Size_X") or r.get("Grid_Size") or ""


def _short(name: str, width: int = 72) -> str:
    return name if len(name) <= width else name[:width - 3] + "..."


def trace(d: str, kernel: str, grid: str | None, last: int) -> str:
    rows = _rows(d, "kernel_trace.csv")
    groups = collections.defaultdict(list)
    for r in rows:
        groups[(r["Kernel_Name"], _grid(r))].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    out = ["%-72s %9s %7s %10s %10s %10s %10s" % ("kernel", "grid_x", "calls", "avg_us", "median_us",
                                                    "min_us", "total_ms")]
    for (name, g), ds in sorted(groups.items(), key=lambda kv: -sum(kv[1]))[:20]:
        out.append("%-72s %9s %7d %10.3f %10.3f %10.3f %10.3f" % (_short(name), g, len(ds), sum(ds) / len(ds),
                                                                  statistics.median(ds), min(ds), sum(ds) / 1e3))
    if grid is not None:
        sel = [ds for (name, g), ds in groups.items() if name.startswith(kernel) and g == grid]
        if not sel:
            seen = sorted(g for (name, g) in groups if name.startswith(kernel))
            raise SystemExit("no %s dispatch at grid %s (grid sizes seen: %s)" % (kernel, grid, seen))
        tail = sel[0][-last:]
        out.append("")
        out.append("%s at grid %s, last %d dispatches: avg %.3f us, median %.3f us" % (
            kernel, grid, len(tail), sum(tail) / len(tail), statistics.median(tail)))
    return "\n".join(out)


def _counter(d: str):
    rows = _rows(d, "counter_collection.csv")
    names = {r["Counter_Name"] for r in rows}
    if len(names) != 1:
        raise SystemExit("expected one counter in %s, found %s" % (d, sorted(names)))
    return names.pop(), rows


def traffic(fetch_dir: str, write_dir: str, grid: str | None, last: int, kernel: str = STEP_KERNEL):
    res = {}
    lines = []
    for d in (fetch_dir, write_dir):
        cname, rows = _counter(d)
        copies = [float(r["Counter_Value"]) for r in rows if r["Kernel_Name"].startswith(COPY_KERNEL)]
        if not copies:
            raise SystemExit("no %s dispatch in %s" % (COPY_KERNEL, d))
        cal = max(copies)                       # KiB as the counter reports it
        scale = (COPY_BYTES / 1024.0) / cal     # true KiB per counter KiB
        if grid is None:
            grids = {r["Grid_Size"] for r in rows if r["Kernel_Name"].startswith(kernel)}
            if len(grids) != 1:
                raise SystemExit("%s ran at grid sizes %s: name one with --grid" % (kernel, sorted(grids)))
            grid = grids.pop()
        vals = [float(r["Counter_Value"]) for r in rows
                if r["Kernel_Name"].startswith(kernel) and r["Grid_Size"] == grid]
        if not vals:
            raise SystemExit("no %s dispatch at grid %s in %s" % (kernel, grid, d))
        tail = vals[-last:]
        mean_kib = sum(tail) / len(tail)
        res[cname] = {"counter_kib_per_dispatch": mean_kib, "copy_counter_kib": cal, "scale": scale,
                      "bytes_per_dispatch": mean_kib * scale * 1024.0, "dispatches": len(tail)}
        lines.append("%-10s copy 64 MiB reads %.1f KiB -> scale %.4f; %s grid %s, last %d dispatches: "
                     "%.1f KiB/dispatch -> %.0f bytes" % (cname, cal, scale, kernel, grid, len(tail), mean_kib,
                                                          mean_kib * scale * 1024.0))
    total = sum(v["bytes_per_dispatch"] for v in res.values())
    doc = {"kernel": kernel, "grid": int(grid), "source_hash": kernel_source_hash(),
           "fetch_bytes": res["FETCH_SIZE"]["bytes_per_dispatch"],
           "write_bytes": res["WRITE_SIZE"]["bytes_per_dispatch"], "traffic_bytes": total,
           "detail": res}
    lines.append("HBM traffic per dispatch: %.0f bytes" % total)
    lines.append("TRAFFIC_JSON " + json.dumps(doc))
    return "\n".join(lines)


def counters(dirs, kernel: str = STEP_KERNEL, grid: str | None = None, last: int = 1000) -> str:
    """Mean of every counter over the last `last` dispatches of `kernel` (at grid
    size `grid`, or its only grid size), from one or more counter runs."""
    out = ["%-36s %14s %10s" % ("counter", "mean/dispatch", "dispatches")]
    for d in dirs:
        rows = _rows(d, "counter_collection.csv")
        sel = [r for r in rows if r["Kernel_Name"].startswith(kernel)]
        g = grid
        if g is None:
            grids = {r["Grid_Size"] for r in sel}
            if len(grids) != 1:
                raise SystemExit("%s ran at grid sizes %s: name one with --grid" % (kernel, sorted(grids)))
            g = grids.pop()
        by = collections.defaultdict(list)
        for r in sel:
            if r["Grid_Size"] == g:
                by[r["Counter_Name"]].append(float(r["Counter_Value"]))
        for name in sorted(by):
            vals = by[name][-last:]
            out.append("%-36s %14.1f %10d" % (name, sum(vals) / len(vals), len(vals)))
    return "\n".join(out)


def read_traffic(path: str):
    """The TRAFFIC_JSON record of a committed summary, or None when the file is
    missing or the step kernel's sources changed since the counters were taken."""
    try:
        with open(path) as f:
            for line in f:
                if line.startswith("TRAFFIC_JSON {"):
                    doc = json.loads(line[len("TRAFFIC_JSON "):])
                    return doc if doc.get("source_hash") == kernel_source_hash() else None
    except OSError:
        return None
    return None


def main():
    p = argparse.ArgumentParser()
    p.add_argument("mode", choices=("trace", "traffic", "counters", "hash"))
    p.add_argument("dirs", nargs="*")
    p.add_argument("--kernel", default=STEP_KERNEL)
    p.add_argument("--grid", default=None)
    p.add_argument("--last", type=int, default=1000)
    a = p.parse_args()
    if a.mode == "hash":
        print(kernel_source_hash())
    elif a.mode == "trace":
        print(trace(a.dirs[0], a.kernel, a.grid, a.last))
    elif a.mode == "counters":
        print(counters(a.dirs, a.kernel, a.grid, a.last))
    else:
        print(traffic(a.dirs[0], a.dirs[1], a.grid, a.last, a.kernel))


if __name__ == "__main__":
    main()
