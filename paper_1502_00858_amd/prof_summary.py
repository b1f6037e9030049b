"""Summaries of rocprofv3 CSV output (kernel trace / stats, FETCH_SIZE and WRITE_SIZE passes).

    python -m paper_1502_00858_amd.prof_summary trace DIR [--between NAME]
                                                # DIR: --kernel-trace --stats -o run
    python -m paper_1502_00858_amd.prof_summary pmc FETCH_DIR WRITE_DIR [--between NAME]

`trace` prints, per kernel, calls, total and average time and the average over dispatches longer
than 5 us (launches whose subbands all stopped their LM runs exit at once), and, for the Cholesky
solve, the wall time of each full solve: from the first kernel of a solve to the end of its last
one (blocked solver: the panel launches + back substitution; one-workgroup solver: one launch).
With --between NAME, only the dispatches that run after the first dispatch of a kernel whose name
contains NAME ends and before the second one starts (bench.py brackets its timed steps of the
learned start with such a kernel).  `pmc` prints per-dispatch FETCH_SIZE / WRITE_SIZE per kernel in MB, scaled by what the counters
read for the 256 MiB device copy that profile_run ends with, and per-solve sums for the Cholesky.
Output is markdown on stdout.
"""
from __future__ import annotations

import collections
import csv
import glob
import os
import sys

COPY_BYTES = 268435456
FULL_US = 5.0


def _short(name: str) -> str:
    name = name.replace("calib::(anonymous namespace)::", "").replace("(anonymous namespace)::", "")
    return name.split("(")[0]


def _one(dirname: str, suffix: str) -> str:
    hits = glob.glob(os.path.join(dirname, "**", "*" + suffix), recursive=True)
    if not hits:
        raise SystemExit(f"no *{suffix} under {dirname}")
    return hits[0]


def trace(dirname: str, between: str | None = None):
    rows = list(csv.DictReader(open(_one(dirname, "kernel_trace.csv"))))
    if between:
        rows, (lo, hi) = _window(rows, between, bounds=True)
        print(f"Window: {len(rows)} dispatches over {(hi - lo) / 1e6:.2f} ms between the first two "
              f"dispatches of {between}.\n")
    per = collections.defaultdict(list)
    seq = []
    for r in rows:
        d = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
        n = _short(r["Kernel_Name"])
        per[n].append(d)
        seq.append((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), n, d))
    total = sum(sum(v) for v in per.values())
    print("| kernel | calls | total ms | avg us | share | calls > 5 us | avg us of those |")
    print("|---|---:|---:|---:|---:|---:|---:|")
    for n, v in sorted(per.items(), key=lambda kv: -sum(kv[1])):
        full = [x for x in v if x > FULL_US]
        print(f"| {n} | {len(v)} | {sum(v) / 1e3:.2f} | {sum(v) / len(v):.1f} | "
              f"{100 * sum(v) / total:.1f}% | {len(full)} | "
              f"{(sum(full) / len(full)) if full else 0:.1f} |")
    # full Cholesky solves: a run of panel launches closed by a back substitution, or one launch
    seq.sort()
    solves, start = [], None
    for s, e, n, d in seq:
        if n == "k_chol_panel":
            if start is None:
                start = (s, d)
            elif d > FULL_US and start[1] <= FULL_US:
                start = (s, d)
        elif n in ("k_chol_backsub", "k_chol_backsub_ring") and start is not None:
            if d > FULL_US:
                solves.append((e - start[0]) / 1e3)
            start = None
        elif n == "k_chol_solve" and d > FULL_US:
            solves.append(d)
    if solves:
        solves.sort()
        print(f"\nFull Cholesky solves: {len(solves)}, wall time per solve: mean "
              f"{sum(solves) / len(solves):.1f} us, median {solves[len(solves) // 2]:.1f} us")


def _window(rows, between, bounds=False):
    """The rows of dispatches that start after the first dispatch of a kernel named like `between`
    ends and end before its second one starts (all rows when between is None); with bounds, also
    the window's (start, end) timestamps."""
    if not between:
        return (rows, None) if bounds else rows
    marks = sorted((int(r["Start_Timestamp"]), int(r["End_Timestamp"])) for r in rows
                   if between in r["Kernel_Name"])
    if len(marks) < 2:
        raise SystemExit(f"fewer than two dispatches of {between}")
    lo, hi = marks[0][1], marks[1][0]
    inside = [r for r in rows if int(r["Start_Timestamp"]) >= lo and int(r["End_Timestamp"]) <= hi]
    return (inside, (lo, hi)) if bounds else inside


def _pmc(dirname: str, between=None):
    path = _one(dirname, "counter_collection.csv")
    rows = list(csv.DictReader(open(path)))
    vals = collections.defaultdict(list)
    copies = [r for r in rows if "copyBuffer" in r["Kernel_Name"]]
    for r in _window(rows, between) + (copies if between else []):
        vals[_short(r["Kernel_Name"])].append(float(r["Counter_Value"]))
    return vals


def pmc(fetch_dir: str, write_dir: str, between=None):
    fv, wv = _pmc(fetch_dir, between), _pmc(write_dir, between)
    if between:
        print(f"Window: the dispatches between the first two dispatches of {between} (the "
              f"calibration copy taken from the whole run).\n")
    copy = [k for k in fv if "copyBuffer" in k]
    if not copy:
        raise SystemExit("no copy kernel in the FETCH_SIZE pass")
    fscale = COPY_BYTES / 1024.0 / max(fv[copy[0]])
    wscale = COPY_BYTES / 1024.0 / max(wv[copy[0]])
    print(f"Calibration: the 256 MiB copy read FETCH_SIZE {max(fv[copy[0]]):.1f} KiB (x{fscale:.4f}), "
          f"WRITE_SIZE {max(wv[copy[0]]):.1f} KiB (x{wscale:.4f}).\n")
    print("| kernel | dispatches | fetch MB/dispatch | write MB/dispatch |")
    print("|---|---:|---:|---:|")
    for n in fv:
        if n in copy:
            continue
        f = sum(fv[n]) / len(fv[n]) * 1024 * fscale / 1e6
        w = (sum(wv[n]) / len(wv[n]) * 1024 * wscale / 1e6) if n in wv else float("nan")
        print(f"| {n} | {len(fv[n])} | {f:.2f} | {w:.2f} |")
    names = ("k_chol_panel", "k_chol_backsub", "k_chol_backsub_ring", "k_chol_solve")
    solves = sum(len(fv.get(n, [])) for n in names[1:])
    if solves:
        tf = sum(sum(fv.get(n, [])) for n in names)
        tw = sum(sum(wv.get(n, [])) for n in names)
        print(f"\nCholesky solve ({solves} solves): fetch {tf / solves * 1024 * fscale / 1e6:.2f} MB + "
              f"write {tw / solves * 1024 * wscale / 1e6:.2f} MB per solve")


if __name__ == "__main__":
    if len(sys.argv) >= 3 and sys.argv[1] == "trace":
        trace(sys.argv[2], sys.argv[4] if len(sys.argv) >= 5 and sys.argv[3] == "--between" else None)
    elif len(sys.argv) >= 4 and sys.argv[1] == "pmc":
        pmc(sys.argv[2], sys.argv[3],
            sys.argv[5] if len(sys.argv) >= 6 and sys.argv[4] == "--between" else None)
    else:
        raise SystemExit(__doc__)
