"""Summaries of rocprofv3 runs of `bench.py --profile-sweeps` (host-side
bookkeeping, no GPU work).

`bench.py --profile-sweeps` runs, after setup and the autotuner, exactly S
timed smoothing sweeps per storage type (and, with --copy-calibration, three
device copies of 256 MiB).  The summaries keep, for every kernel name that
matches a pattern, only its last S dispatches, so that launches of the
autotuner (same kernels, other grids) are excluded:

  python -m paper_2510_00998_amd.profiling times  <kernel_trace.csv> <S> <regex>
  python -m paper_2510_00998_amd.profiling counter <counter_collection.csv> <S> <regex>

`times` prints the mean duration per dispatch; `counter` the mean counter
value per dispatch (KiB for FETCH_SIZE / WRITE_SIZE) and the copy kernel's
value for calibration.
"""
from __future__ import annotations

import csv
import re
import statistics
import sys
from collections import defaultdict


def _col(header, *names):
    for n in names:
        for i, h in enumerate(header):
            if h.strip().lower() == n.lower():
                return i
    raise KeyError(f"none of {names} in {header}")


def _rows(path):
    with open(path, newline="") as f:
        r = csv.reader(f)
        header = next(r)
        return header, list(r)


def dispatch_times(path, last, pattern):
    """{kernel name: (dispatches kept, mean duration in us)} over the last
    `last` dispatches of every kernel whose name matches `pattern`."""
    header, rows = _rows(path)
    kn = _col(header, "Kernel_Name")
    t0 = _col(header, "Start_Timestamp")
    t1 = _col(header, "End_Timestamp")
    di = _col(header, "Dispatch_Id", "Correlation_Id")
    rx = re.compile(pattern)
    per = defaultdict(list)
    for row in rows:
        if rx.search(row[kn]):
            per[row[kn]].append((int(row[di]), (int(row[t1]) - int(row[t0])) * 1e-3))
    out = {}
    for k, v in per.items():
        v.sort()
        kept = [d for _, d in v[-last:]]
        out[k] = (len(kept), statistics.fmean(kept))
    return out


def dispatch_counter(path, last, pattern, counter):
    """{kernel name: (dispatches kept, mean value)} of `counter` over the last
    `last` dispatches of every matching kernel."""
    header, rows = _rows(path)
    kn = _col(header, "Kernel_Name")
    di = _col(header, "Dispatch_Id", "Correlation_Id")
    cn = _col(header, "Counter_Name")
    cv = _col(header, "Counter_Value")
    rx = re.compile(pattern)
    per = defaultdict(dict)
    for row in rows:
        if row[cn].strip() == counter and rx.search(row[kn]):
            d = int(row[di])
            per[row[kn]][d] = per[row[kn]].get(d, 0.0) + float(row[cv])  # summed over dimensions
    out = {}
    for k, v in per.items():
        kept = [v[d] for d in sorted(v)[-last:]]
        out[k] = (len(kept), statistics.fmean(kept))
    return out


def main(argv):
    mode, path, last, pattern = argv[0], argv[1], int(argv[2]), argv[3]
    if mode == "times":
        res = dispatch_times(path, last, pattern)
        print("| kernel | dispatches | mean duration [us] |")
        print("|---|---|---|")
        for k, (c, m) in sorted(res.items()):
            print(f"| `{k[:110]}` | {c} | {m:.2f} |")
    else:
        counter = argv[4]
        res = dispatch_counter(path, last, pattern, counter)
        print(f"| kernel | dispatches | {counter} [KiB] per dispatch |")
        print("|---|---|---|")
        for k, (c, m) in sorted(res.items()):
            print(f"| `{k[:110]}` | {c} | {m:.1f} |")


if __name__ == "__main__":
    main(sys.argv[1:])
