"""Overlap figures (Sec. V-F: CT, TC, CC, TOT) from a rocprofv3 timeline,
for checking the library's own event-based figures.

Reads the CSV files a run of
  DAGRT_ROCTX=1 rocprofv3 --kernel-trace --memory-copy-trace --marker-trace --output-format csv -d DIR -o p -- ...
left in DIR: every kernel dispatch whose name contains one of --kernels is a
computation interval, every memory copy a transfer interval (the copy
kernel's dispatches count as transfers when their name matches
--copy-kernels).  The roctx ranges of the library (one per GPU task, named
"dagrt task <id> <what> stream <s> waits <n>") give the number of tasks
submitted and, per run, the window: intervals before the first task (the
input uploads) are left out, the rest grouped into runs by the largest gaps
between the roctx ranges of consecutive runs (--runs).

Usage: python -m paper_2012_09646_amd.trace_overlap DIR --kernels bs_call --copy-kernels k_copy_bytes \
           --runs 3 --tasks-per-run 30
Prints one JSON line.
"""

import argparse
import csv
import glob
import json
import os

from . import metrics as M


def _rows(d, suffix):
    paths = glob.glob(os.path.join(d, "*" + suffix))
    if not paths:
        return []
    with open(paths[0]) as f:
        return list(csv.DictReader(f))


def intervals(d, kernels, copy_kernels):
    """[(kind, start_ns, end_ns)] of the matching kernels ('C'), copy kernels
    and memory copies ('T')."""
    out = []
    for r in _rows(d, "kernel_trace.csv"):
        name = r["Kernel_Name"]
        a, b = int(r["Start_Timestamp"]), int(r["End_Timestamp"])
        if any(k in name for k in copy_kernels):
            out.append(("T", a, b))
        elif any(k in name for k in kernels):
            out.append(("C", a, b))
    for r in _rows(d, "memory_copy_trace.csv"):
        out.append(("T", int(r["Start_Timestamp"]), int(r["End_Timestamp"])))
    return sorted(out, key=lambda t: t[1])


def task_ranges(d):
    """Start/end (ns) of the library's per-task roctx ranges, in order."""
    out = []
    for r in _rows(d, "marker_api_trace.csv"):
        msg = r.get("Function") or r.get("Message") or ""
        if msg.startswith("dagrt task"):
            out.append((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), msg))
    return sorted(out)


def split_runs(ivs, ranges, runs, tasks_per_run=0):
    """Group intervals into `runs` runs.  The runs' first tasks are every
    `tasks_per_run`-th roctx range when that is given, else the ranges that
    follow the `runs - 1` largest gaps between consecutive task submissions;
    each run owns the intervals that start after its first submission."""
    if not ranges:
        return [ivs]
    if runs <= 1 or len(ranges) < runs:
        return [[iv for iv in ivs if iv[1] >= ranges[0][0]]]
    if tasks_per_run:
        starts = [ranges[i][0] for i in range(0, min(len(ranges), runs * tasks_per_run), tasks_per_run)]
    else:
        gaps = sorted(range(1, len(ranges)), key=lambda i: ranges[i][0] - ranges[i - 1][1], reverse=True)[:runs - 1]
        starts = [ranges[0][0]] + sorted(ranges[i][0] for i in gaps)
    groups = [[] for _ in starts]
    for iv in ivs:
        if iv[1] < starts[0]:
            continue  # before the first task (uploads)
        k = max(i for i, s in enumerate(starts) if iv[1] >= s)
        groups[k].append(iv)
    return groups


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("dir")
    ap.add_argument("--kernels", default="", help="comma-separated substrings of computation kernel names")
    ap.add_argument("--copy-kernels", default="", help="comma-separated substrings of copy kernel names")
    ap.add_argument("--runs", type=int, default=1)
    ap.add_argument("--tasks-per-run", type=int, default=0, help="GPU tasks per run (splits the runs exactly)")
    a = ap.parse_args()
    ks = [k for k in a.kernels.split(",") if k]
    cks = [k for k in a.copy_kernels.split(",") if k]
    ivs = intervals(a.dir, ks, cks)
    ranges = task_ranges(a.dir)
    per_run = []
    for g in split_runs(ivs, ranges, a.runs, a.tasks_per_run):
        if not g:
            continue
        o = M.overlap([(k, s / 1e6, e / 1e6) for k, s, e in g])
        o["span_ms"] = (max(e for _, _, e in g) - min(s for _, s, _ in g)) / 1e6
        o["kernels"] = sum(1 for k, _, _ in g if k == "C")
        o["transfers"] = sum(1 for k, _, _ in g if k == "T")
        per_run.append(o)
    print(json.dumps({"dir": a.dir, "tasks_submitted": len(ranges), "runs": per_run}), flush=True)


if __name__ == "__main__":
    main()
