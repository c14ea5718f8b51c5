"""Summaries of rocprofv3 output for the benchmark (profiles/*.txt).

    python -m paper_1507_01926_amd.profiling kernels <trace dir> <title> [<kernel> [<stride>]]
    python -m paper_1507_01926_amd.profiling traffic <fetch dir> <write dir> <kernel> <workload> <probe MiB>

`kernels` condenses a `--kernel-trace --output-format csv` run into one
line per kernel (calls, total, average) over the dispatches of the last
solve of the run (from its last k_init_state dispatch on).  `traffic` turns
two `--pmc FETCH_SIZE` / `--pmc WRITE_SIZE` runs into HBM bytes per launch
of one kernel over the last solve, each counter scaled by what it reads for
the benchmark's device copy of known size (--copy-probe-mib: that many MiB
read and written, the last device copy before the solve), in the key: value
form that bench.py reads back.
"""
from __future__ import annotations

import collections
import csv
import glob
import hashlib
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))


def source_sha() -> str:
    """sha256 over the library's HIP sources (the figures describe these)."""
    h = hashlib.sha256()
    d = os.path.join(HERE, "csrc")
    for name in sorted(os.listdir(d)):
        if name.endswith((".hip", ".h")):
            with open(os.path.join(d, name), "rb") as fh:
                h.update(name.encode() + b"\0" + fh.read())
    return h.hexdigest()


def _rows(root: str, suffix: str):
    files = sorted(glob.glob(os.path.join(root, "**", "*" + suffix), recursive=True))
    for f in files:
        with open(f, newline="") as fh:
            yield from csv.DictReader(fh)


def _order(r) -> int:
    """Launch order of a dispatch row (dispatch ids grow in launch order)."""
    for k in ("Dispatch_Id", "Correlation_Id", "Start_Timestamp"):
        if r.get(k):
            return int(r[k])
    return 0


def _split_last_solve(rows):
    """(rows before the last solve, rows of the last solve, solves seen): a
    solve starts with its k_init_state dispatch."""
    rows = sorted(rows, key=_order)
    starts = [i for i, r in enumerate(rows) if "k_init_state" in r["Kernel_Name"]]
    if not starts:
        return [], rows, 0
    return rows[:starts[-1]], rows[starts[-1]:], len(starts)


def _last_solve(rows):
    _, last, n = _split_last_solve(rows)
    return last, n


def kernel_summary(trace_dir: str, title: str, sampled: str = "", stride: int = 16) -> str:
    """Per-kernel table of the last solve.  With `sampled`, also the average
    duration of that kernel's launches 0, stride, 2*stride, ... of the solve
    (the ones the benchmark brackets with HIP events) and of the others."""
    rows, solves = _last_solve(list(_rows(trace_dir, "kernel_trace.csv")))
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    agg = collections.defaultdict(lambda: [0, 0])
    for r in rows:
        a = agg[r["Kernel_Name"]]
        a[0] += 1
        a[1] += int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
    span = (int(rows[-1]["End_Timestamp"]) - int(rows[0]["Start_Timestamp"])) / 1e6
    busy = sum(v[1] for v in agg.values()) / 1e6
    out = [f"# {title}",
           f"# last solve of the run ({solves} solves traced): {len(rows)} dispatches, wall span {span:.1f} ms "
           f"under the trace, kernels busy {busy:.1f} ms",
           "# kernel" + " " * 62 + "calls   total_ms    avg_us    pct"]
    for k, (c, t) in sorted(agg.items(), key=lambda x: -x[1][1]):
        out.append(f"{k[:68]:68s} {c:8d} {t / 1e6:10.2f} {t / 1e3 / c:9.2f} {100 * t / 1e6 / busy:6.2f}")
    if sampled:
        d = [int(r["End_Timestamp"]) - int(r["Start_Timestamp"]) for r in rows if sampled in r["Kernel_Name"]]
        on = [x for i, x in enumerate(d) if i % stride == 0]
        off = [x for i, x in enumerate(d) if i % stride != 0]
        if on and off:
            out.append(f"# {sampled}: launches 0, {stride}, {2 * stride}, ... of the solve (the ones the benchmark "
                       f"brackets with HIP events): {len(on)} launches, avg {sum(on) / len(on) / 1e3:.2f} us; "
                       f"the other {len(off)}: avg {sum(off) / len(off) / 1e3:.2f} us")
    return "\n".join(out) + "\n"


def _counter(root: str, name: str, kernel: str):
    """(per-dispatch values of `kernel` in the last solve, value of the copy
    probe) of counter `name`, in the counter's unit (KiB)."""
    rows = [r for r in _rows(root, "counter_collection.csv") if r.get("Counter_Name") == name]
    before, last, _ = _split_last_solve(rows)
    # the probe copy is the last device copy launched before the solve
    probe = [float(r["Counter_Value"]) for r in before if "copyBuffer" in r["Kernel_Name"]]
    vals = [float(r["Counter_Value"]) for r in last if kernel in r["Kernel_Name"]]
    sym = next((r["Kernel_Name"] for r in last if kernel in r["Kernel_Name"]), kernel)
    return vals, (probe[-1] if probe else None), sym


def traffic_summary(fetch_dir: str, write_dir: str, kernel: str, workload: str, probe_mib: int,
                    command: str) -> str:
    f, fp, sym = _counter(fetch_dir, "FETCH_SIZE", kernel)
    w, wp, _ = _counter(write_dir, "WRITE_SIZE", kernel)
    probe_kib = probe_mib * 1024.0
    fs = probe_kib / fp if fp else 1.0
    ws = probe_kib / wp if wp else 1.0
    per_launch = 1024.0 * (fs * sum(f) + ws * sum(w)) / max(1, len(f))
    return "\n".join([
        f"# HBM traffic of {sym} on the {workload} workload (one solve), from two rocprofv3 counter runs:",
        f"#   {command.replace('PMC', 'FETCH_SIZE')}",
        f"#   {command.replace('PMC', 'WRITE_SIZE')}",
        "# (repository root, TMPDIR=/tmp).  Figures cover the dispatches of the last solve.  Counters are KiB",
        f"# per dispatch, each scaled by what it reads for a device copy of {probe_mib} MiB in the same run",
        f"# ({probe_mib} MiB read and {probe_mib} MiB written).",
        f"kernel: {kernel}",
        f"kernel_symbol: {sym}",
        f"workload: {workload}",
        f"source_sha256: {source_sha()}",
        f"dispatches: {len(f)}",
        f"fetch_kib_total: {sum(f):.1f}",
        f"write_kib_total: {sum(w):.1f}",
        f"copy_probe_fetch_kib: {fp}",
        f"copy_probe_write_kib: {wp}",
        f"fetch_scale: {fs:.4f}",
        f"write_scale: {ws:.4f}",
        f"hbm_bytes_per_launch: {per_launch:.0f}",
    ]) + "\n"


if __name__ == "__main__":
    a = sys.argv[1:]
    if a[:1] == ["kernels"]:
        sys.stdout.write(kernel_summary(a[1], a[2], *(a[3:4]), *(int(x) for x in a[4:5])))
    elif a[:1] == ["traffic"]:
        sys.stdout.write(traffic_summary(a[1], a[2], a[3], a[4], int(a[5]), a[6] if len(a) > 6 else ""))
    else:
        print(__doc__)
