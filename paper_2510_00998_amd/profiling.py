"""Summaries of rocprofv3 runs of `bench.py --profile-sweeps` (host-side
bookkeeping, no GPU work).

`bench.py --profile-sweeps` runs, after setup and the autotuner, exactly S
timed smoothing sweeps per storage type (and, with --copy-calibration, three
device copies of 256 MiB).  The summaries keep, for every kernel name that
matches a pattern, only its last S dispatches, so that launches of the
autotuner (same kernels, other grids) are excluded:

  python -m paper_2510_00998_amd.profiling times  <kernel_trace.csv> <S> <regex>
  python -m paper_2510_00998_amd.profiling counter <counter_collection.csv> <S> <regex>
  python -m paper_2510_00998_amd.profiling summary <trace> <fetch> <write> <S> <keys json> <sources> <title> <command> [<extra json>]
  python -m paper_2510_00998_amd.profiling sq <counter_collection.csv> <S> <keys json> <title> <command>
  python -m paper_2510_00998_amd.profiling timeline <kernel_trace.csv> <marker regex> <title> <command>

`times` prints the mean duration per dispatch; `counter` the mean counter
value per dispatch (KiB for FETCH_SIZE / WRITE_SIZE) and the copy kernel's
value for calibration; `timeline` the kernels of one solver iteration of a
`bench.py --profile-solve` trace, with the idle gaps between them.
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


def dispatch_times(path, last, pattern, skip=0):
    """{kernel name: (dispatches kept, mean duration in us)} over the last
    `last` dispatches (before the final `skip` ones) of every kernel whose
    name matches `pattern`."""
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
        kept = [d for _, d in v[len(v) - last - skip:len(v) - skip]]
        if kept:
            out[k] = (len(kept), statistics.fmean(kept))
    return out


def dispatch_counter(path, last, pattern, counter, skip=0):
    """{kernel name: (dispatches kept, mean value)} of `counter` over the last
    `last` dispatches (before the final `skip` ones) of every matching
    kernel."""
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
        ids = sorted(v)
        kept = [v[d] for d in ids[len(ids) - last - skip:len(ids) - skip]]
        if kept:
            out[k] = (len(kept), statistics.fmean(kept))
    return out


def summary(trace, fetch, write, last, keys, sources, title, command, extra=None):
    """Markdown summary of one --profile-sweeps workload: per key (a regex
    over kernel names, or [regex, skip] to leave out the final `skip`
    dispatches of the matching kernels, e.g. a second timed series of the
    same kernel) the mean duration and copy-calibrated HBM bytes of the last
    `last` dispatches of every matching kernel, and their sums; the copy
    calibration divides the known 256 MiB of the last three copy dispatches
    by their counter readings."""
    import hashlib
    import json
    import os
    keys = json.loads(keys)
    cf = dispatch_counter(fetch, 3, r"copyBuffer", "FETCH_SIZE")
    cw = dispatch_counter(write, 3, r"copyBuffer", "WRITE_SIZE")
    kf = 262144.0 / list(cf.values())[0][1]
    kw = 262144.0 / list(cw.values())[0][1]
    csrc = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")
    h = hashlib.sha256()
    for src in sources.split(","):
        h.update(open(os.path.join(csrc, src), "rb").read())
    out = [f"# {title}", "", "Commands (from /tmp with TMPDIR=/tmp, repository at $R; each counter in a run of its own):",
           ""] + ["    " + c for c in command.split(" ;; ")] + [
        "", f"Per key, the last {last} dispatches of each matching kernel are kept (the timed sweeps; autotuner and "
            "setup launches of the same kernels come earlier; where a key skips dispatches, a later timed series of "
            "the same kernel is left out).  Copy calibration: a 256 MiB device copy reads FETCH_SIZE = "
            f"{list(cf.values())[0][1]:.1f} KiB and WRITE_SIZE = {list(cw.values())[0][1]:.1f} KiB per dispatch, so "
            f"FETCH_SIZE is scaled by {kf:.4f} and WRITE_SIZE by {kw:.4f} to give bytes.", "",
        "| key | kernel | dispatches | mean duration [us] | read [MB] | write [MB] | total [MB] |",
        "|---|---|---|---|---|---|---|"]
    tot = {}
    for key, spec in keys.items():
        rx, skip = (spec, 0) if isinstance(spec, str) else (spec[0], int(spec[1]))
        t = dispatch_times(trace, last, rx, skip)
        f = dispatch_counter(fetch, last, rx, "FETCH_SIZE", skip)
        w = dispatch_counter(write, last, rx, "WRITE_SIZE", skip)
        a = tot.setdefault(key, [0.0, 0.0])
        for k in sorted(t):
            rd = f[k][1] * 1024 * kf if k in f else float("nan")
            wr = w[k][1] * 1024 * kw if k in w else float("nan")
            out.append(f"| {key} | `{k[:90]}` | {t[k][0]} | {t[k][1]:.2f} | {rd / 1e6:.2f} | {wr / 1e6:.2f} | "
                       f"{(rd + wr) / 1e6:.2f} |")
            a[0] += t[k][1]
            a[1] += rd + wr
    out += ["", "| key | summed mean duration [us] | summed bytes per launch |", "|---|---|---|"]
    for key, (dur, by) in tot.items():
        out.append(f"| {key} | {dur:.2f} | {by:.0f} |")
    out += ["", "Machine-readable (bench.py reads these while the kernel sources hash to the value below):", "",
            f"    source_sha256: {h.hexdigest()}"]
    for key, (dur, by) in tot.items():
        out.append(f"    traffic_bytes_{key}: {by:.0f}")
        out.append(f"    mean_duration_us_{key}: {dur:.3f}")
    for k, v in json.loads(extra or "{}").items():  # launch configuration the counters belong to
        out.append(f"    {k}: {v}")
    print("\n".join(out))


# SQ counters of one pass (at most 8) and the derived activity of a kernel:
# busy = SQ_BUSY_CYCLES / 32 shader engines (cycles the kernel kept the
# sequencers busy); VALU and LDS busy = 4 x SQ_ACTIVE_INST_* (quad-cycles)
# / (1024 SIMDs x busy); MFMA busy = SQ_VALU_MFMA_BUSY_CYCLES / (1024 SIMDs x
# busy).
SQ_COUNTERS = ["SQ_WAVES", "SQ_BUSY_CYCLES", "SQ_ACTIVE_INST_VALU", "SQ_ACTIVE_INST_LDS", "SQ_INSTS_VALU",
               "SQ_INSTS_MFMA", "SQ_VALU_MFMA_BUSY_CYCLES", "SQ_INSTS_LDS"]


def sq(path, last, keys, title, command):
    """Markdown table of the SQ_COUNTERS pass: per key (label -> regex that
    matches one kernel name) the mean of its last `last` dispatches."""
    import json
    keys = json.loads(keys)
    out = [f"# {title}", "", "Command (from /tmp with TMPDIR=/tmp, repository at $R):", ""] + \
        ["    " + c for c in command.split(" ;; ")] + [
        "", f"Mean over the last {last} dispatches of each kernel.  busy = SQ_BUSY_CYCLES / 32 shader engines; "
            "VALU (LDS) busy = 4 x SQ_ACTIVE_INST_VALU (_LDS) / (1024 SIMDs x busy); MFMA busy = "
            "SQ_VALU_MFMA_BUSY_CYCLES / (1024 SIMDs x busy).", "",
        "| kernel | " + " | ".join(c[3:] for c in SQ_COUNTERS) + " | busy [cycles] | VALU busy | LDS busy | MFMA busy |",
        "|---" * (len(SQ_COUNTERS) + 5) + "|"]
    for label, rx in keys.items():
        vals = {}
        for c in SQ_COUNTERS:
            r = dispatch_counter(path, last, rx, c)
            if len(r) != 1:
                raise SystemExit(f"{label}: regex {rx} matches {len(r)} kernels for {c}")
            vals[c] = list(r.values())[0][1]
        busy = vals["SQ_BUSY_CYCLES"] / 32
        v = 4 * vals["SQ_ACTIVE_INST_VALU"] / (1024 * busy)
        lds = 4 * vals["SQ_ACTIVE_INST_LDS"] / (1024 * busy)
        mf = vals["SQ_VALU_MFMA_BUSY_CYCLES"] / (1024 * busy)
        out.append(f"| {label} | " + " | ".join(f"{vals[c]:.0f}" for c in SQ_COUNTERS) +
                   f" | {busy:.0f} | {100 * v:.0f}% | {100 * lds:.0f}% | {100 * mf:.0f}% |")
    print("\n".join(out))


def _short(name):
    """Kernel name without its parameter list and anonymous namespaces."""
    depth = 0
    if name.endswith(")"):
        for j in range(len(name) - 1, -1, -1):
            if name[j] == ")":
                depth += 1
            elif name[j] == "(":
                depth -= 1
                if depth == 0:
                    name = name[:j]
                    break
    return name.replace("(anonymous namespace)::", "").replace("void ", "")


def timeline(path, marker, title, command):
    """One iteration of a solve from a kernel trace: the dispatches after the
    second-to-last dispatch of the kernel matching `marker` up to and
    including the last one (the last complete iteration of the last solve),
    in start order, with their durations and the idle gaps between them."""
    header, rows = _rows(path)
    kn = _col(header, "Kernel_Name")
    t0 = _col(header, "Start_Timestamp")
    t1 = _col(header, "End_Timestamp")
    ev = sorted((int(r[t0]), int(r[t1]), r[kn]) for r in rows)
    rx = re.compile(marker)
    marks = [i for i, e in enumerate(ev) if rx.search(e[2])]
    if len(marks) < 2:
        raise SystemExit(f"fewer than two dispatches match {marker!r}")
    a, b = marks[-2], marks[-1]
    it = ev[a + 1:b + 1]
    start = ev[a][1]
    print(f"# {title}\n")
    print("Command (from /tmp with TMPDIR=/tmp, repository at $R):\n")
    for c in command.split(" && "):
        print(f"    {c}")
    print()
    print(f"One iteration: the {len(it)} dispatches after the second-to-last `{marker}` dispatch of the trace up to "
          "and including the last one, in start order; gap = idle time since the previous dispatch ended.\n")
    print("| # | kernel | start [us] | duration [us] | gap before [us] |")
    print("|---|---|---|---|---|")
    prev = start
    busy = gaps = 0.0
    per = defaultdict(lambda: [0, 0.0])
    for i, (s0, s1, k) in enumerate(it):
        d = (s1 - s0) * 1e-3
        g = max(0.0, (s0 - prev) * 1e-3)
        busy += d
        gaps += g
        nm = _short(k)
        per[nm][0] += 1
        per[nm][1] += d
        print(f"| {i} | `{nm[:100]}` | {(s0 - start) * 1e-3:.1f} | {d:.1f} | {g:.1f} |")
        prev = max(prev, s1)
    span = (it[-1][1] - start) * 1e-3
    print(f"\nIteration span {span:.1f} us: kernels {busy:.1f} us, idle gaps {gaps:.1f} us.\n")
    print("| kernel | dispatches | total [us] |")
    print("|---|---|---|")
    for nm, (c, t) in sorted(per.items(), key=lambda kv: -kv[1][1]):
        print(f"| `{nm[:100]}` | {c} | {t:.1f} |")


def main(argv):
    if argv[0] == "timeline":
        # timeline <kernel_trace.csv> <marker regex> <title> <command>
        timeline(argv[1], argv[2], argv[3], argv[4])
        return
    if argv[0] == "sq":
        # sq <counter_collection.csv> <last> <keys json> <title> <command>
        sq(argv[1], int(argv[2]), argv[3], argv[4], argv[5])
        return
    if argv[0] == "summary":
        # summary <trace.csv> <fetch.csv> <write.csv> <last> <keys json> <sources> <title> <command> [<extra json>]
        summary(argv[1], argv[2], argv[3], int(argv[4]), argv[5], argv[6], argv[7], argv[8],
                argv[9] if len(argv) > 9 else None)
        return
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
