"""Summarise rocprofv3 CSV output for the library's kernels.

    python -m paper_1304_4661_amd.rocprof_summary stats DIR
        per-kernel calls / total / average duration from a --kernel-trace
        --stats run (DIR/*_kernel_stats.csv)
    python -m paper_1304_4661_amd.rocprof_summary traffic KERNEL FETCH_DIR WRITE_DIR
                                                   CFETCH_DIR CWRITE_DIR COPY_BYTES
        average FETCH_SIZE / WRITE_SIZE (KiB per dispatch) of KERNEL, scaled by
        what the same counters read for a device copy of COPY_BYTES bytes
        (read COPY_BYTES, write COPY_BYTES), as HBM bytes per launch;
        with LAST after COPY_BYTES only the last LAST dispatches of KERNEL count
    python -m paper_1304_4661_amd.rocprof_summary window KERNEL LAST DIR
        calls / total / average duration of the last LAST dispatches whose
        name contains KERNEL, from a --kernel-trace run (DIR/*_kernel_trace.csv)
    python -m paper_1304_4661_amd.rocprof_summary counters DIR
        every counter of a --pmc run summed over its dispatches
        (DIR/*_counter_collection.csv), with the number of dispatches
    python -m paper_1304_4661_amd.rocprof_summary busy DIR
        for every build in a --kernel-trace run (from its k_validate_graph
        dispatch to its k_final_copy), the span and the time some kernel ran
        (dispatch intervals merged): how much the host-driven loop leaves
        the device idle
"""
from __future__ import annotations

import csv
import glob
import json
import os
import sys


def _rows(d, suffix):
    fs = glob.glob(os.path.join(d, f"*{suffix}"))
    if not fs:
        raise FileNotFoundError(f"no *{suffix} in {d}")
    with open(fs[0]) as f:
        return list(csv.DictReader(f))


def stats(d):
    out = []
    for r in _rows(d, "_kernel_stats.csv"):
        out.append((r["Name"], int(r["Calls"]), float(r["TotalDurationNs"]),
                    float(r["AverageNs"]), float(r["Percentage"])))
    return out


def counter_per_dispatch(d, kernel_substr, counter, last=None):
    rows = [r for r in _rows(d, "_counter_collection.csv")
            if kernel_substr in r["Kernel_Name"] and r["Counter_Name"] == counter]
    rows.sort(key=lambda r: int(r["Dispatch_Id"]))
    if last:
        rows = rows[-last:]
    vals = [float(r["Counter_Value"]) for r in rows]
    return (sum(vals) / len(vals), len(vals)) if vals else (None, 0)


def window(d, kernel_substr, last):
    """(calls, total ns, average ns) of the last `last` dispatches of the
    kernels whose name contains kernel_substr, in start order."""
    rows = [r for r in _rows(d, "_kernel_trace.csv") if kernel_substr in r["Kernel_Name"]]
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    rows = rows[-last:]
    ns = [int(r["End_Timestamp"]) - int(r["Start_Timestamp"]) for r in rows]
    return len(ns), float(sum(ns)), (sum(ns) / len(ns)) if ns else None


def copy_kib(d, counter):
    """The largest per-dispatch value of the counter in a copy-probe run (the
    copy kernel dominates every other dispatch there)."""
    vals = [float(r["Counter_Value"]) for r in _rows(d, "_counter_collection.csv")
            if r["Counter_Name"] == counter]
    return max(vals) if vals else None


def traffic(kernel, fdir, wdir, cfdir, cwdir, copy_bytes, last=None):
    f, nf = counter_per_dispatch(fdir, kernel, "FETCH_SIZE", last)
    w, nw = counter_per_dispatch(wdir, kernel, "WRITE_SIZE", last)
    cf, cw = copy_kib(cfdir, "FETCH_SIZE"), copy_kib(cwdir, "WRITE_SIZE")
    kf = copy_bytes / (cf * 1024.0)  # true bytes per counted byte (reads)
    kw = copy_bytes / (cw * 1024.0)  # (writes)
    return {
        "kernel": kernel, "dispatches": nf,
        "fetch_kib_per_dispatch": f, "write_kib_per_dispatch": w,
        "copy_fetch_kib": cf, "copy_write_kib": cw, "copy_bytes": copy_bytes,
        "fetch_scale": kf, "write_scale": kw,
        "bytes_per_launch": f * 1024.0 * kf + w * 1024.0 * kw,
    }


def counters(d):
    tot, cnt = {}, {}
    for r in _rows(d, "_counter_collection.csv"):
        k = r["Counter_Name"]
        tot[k] = tot.get(k, 0.0) + float(r["Counter_Value"])
        cnt[k] = cnt.get(k, 0) + 1
    return {k: (tot[k], cnt[k]) for k in sorted(tot)}


def busy(d):
    ev = sorted((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), r["Kernel_Name"])
                for r in _rows(d, "_kernel_trace.csv"))
    starts = [i for i, e in enumerate(ev) if "k_validate_graph" in e[2]]
    out = []
    for j, a in enumerate(starts):
        seg = ev[a:starts[j + 1] if j + 1 < len(starts) else len(ev)]
        ends = [i for i, e in enumerate(seg) if "k_final_copy" in e[2]]
        if not ends:
            continue
        seg = seg[:ends[0] + 1]
        run, cs, ce = 0, seg[0][0], seg[0][1]
        for s, e, _ in seg[1:]:
            if s > ce:
                run += ce - cs
                cs, ce = s, e
            else:
                ce = max(ce, e)
        run += ce - cs
        out.append((seg[-1][1] - seg[0][0], run))
    return out


def main(argv):
    if argv[0] == "stats":
        rows = stats(argv[1])
        print(f"{'kernel':70s} {'calls':>7s} {'total ms':>10s} {'avg us':>10s} {'%':>6s}")
        for name, calls, tot, avg, pct in rows:
            print(f"{name[:70]:70s} {calls:7d} {tot / 1e6:10.3f} {avg / 1e3:10.2f} {pct:6.2f}")
    elif argv[0] == "traffic":
        last = int(argv[7]) if len(argv) > 7 else None
        print(json.dumps(traffic(argv[1], argv[2], argv[3], argv[4], argv[5], float(argv[6]),
                                 last), indent=1))
    elif argv[0] == "window":
        calls, tot, avg = window(argv[3], argv[1], int(argv[2]))
        print(f"{argv[1]}: last {calls} dispatches, {tot / 1e6:.3f} ms, {avg / 1e3:.2f} us "
              "per launch")
    elif argv[0] == "counters":
        for k, (v, c) in counters(argv[1]).items():
            print(f"{k:26s} {v:20.0f}  ({c} dispatches)")
    elif argv[0] == "busy":
        rows = busy(argv[1])
        for span, run in rows:
            print(f"  span {span / 1e6:9.1f} ms, kernels {run / 1e6:9.1f} ms, busy {run / span:.3f}")
        fr = [run / span for span, run in rows]
        if fr:
            print(f"  {len(rows)} builds, busy {min(fr):.3f} .. {max(fr):.3f}")
    else:
        raise SystemExit(__doc__)


if __name__ == "__main__":
    main(sys.argv[1:])
