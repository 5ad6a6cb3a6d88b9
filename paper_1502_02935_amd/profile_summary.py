"""Summarise rocprofv3 CSV output (kernel trace/stats, FETCH_SIZE/WRITE_SIZE
counter runs) of this library into a short text table.

    python -m paper_1502_02935_amd.profile_summary stats  <kernel_stats.csv>
    python -m paper_1502_02935_amd.profile_summary trace  <kernel_trace.csv>
    python -m paper_1502_02935_amd.profile_summary counter <counter_collection.csv> [copy_bytes]
    python -m paper_1502_02935_amd.profile_summary markers <marker_api_trace.csv>

The counter mode reports the per-kernel average of every counter per
dispatch (FETCH_SIZE and WRITE_SIZE are in KiB), and, for a single-counter
run with copy_bytes given, the ratio of the plain copy kernel's reading to
its known traffic (the scale factor for the others).
"""
from __future__ import annotations

import collections
import csv
import sys


def stats(path):
    rows = list(csv.DictReader(open(path)))
    print("%-28s %8s %12s %12s %7s" % ("kernel", "calls", "avg_us", "total_ms", "pct"))
    for r in rows:
        print("%-28s %8s %12.1f %12.3f %7.2f" % (r["Name"][:28], r["Calls"],
                                                 float(r["AverageNs"]) / 1e3,
                                                 float(r["TotalDurationNs"]) / 1e6,
                                                 float(r["Percentage"])))


def trace(path):
    """Average duration per (kernel, grid) in dispatch order groups."""
    rows = list(csv.DictReader(open(path)))
    agg = collections.OrderedDict()
    for r in rows:
        name = r.get("Kernel_Name", r.get("Name", "?"))
        key = (name[:60], r.get("Grid_Size_X", r.get("Grid_Size", "")))
        d = int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
        agg.setdefault(key, []).append(d)
    print("%-60s %10s %6s %12s" % ("kernel", "grid", "calls", "avg_us"))
    for (k, gsz), v in agg.items():
        print("%-60s %10s %6d %12.1f" % (k, gsz, len(v), sum(v) / len(v) / 1e3))


def counter(path, copy_bytes=None):
    rows = list(csv.DictReader(open(path)))
    per = collections.OrderedDict()
    for r in rows:
        per.setdefault(r["Counter_Name"], collections.OrderedDict()).setdefault(
            r["Kernel_Name"][:40], []).append(float(r["Counter_Value"]))
    for cname, ks in per.items():
        print("counter %s (per dispatch%s)" % (cname, "; KiB" if "SIZE" in cname else ""))
        print("%-40s %8s %16s" % ("kernel", "calls", "average"))
        for k, v in ks.items():
            print("%-40s %8d %16.1f" % (k, len(v), sum(v) / len(v)))
    per = next(iter(per.values())) if len(per) == 1 else {}
    if copy_bytes:
        for k, v in per.items():
            if "elementwise" in k or "copy" in k.lower():
                avg = max(v)
                print("copy kernel %s: %.1f KiB read vs %.1f KiB known -> factor %.4f" % (
                    k, avg, copy_bytes / 1024.0, avg / (copy_bytes / 1024.0)))


def markers(path):
    """Count and mean duration of each roctx range (host-side spans)."""
    rows = list(csv.DictReader(open(path)))
    agg = collections.OrderedDict()
    for r in rows:
        name = r.get("Function") or r.get("Message") or r.get("Name") or "?"
        d = int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
        agg.setdefault(name[:40], []).append(d)
    print("%-40s %8s %12s %12s" % ("range", "count", "avg_us", "total_ms"))
    for k, v in agg.items():
        print("%-40s %8d %12.1f %12.3f" % (k, len(v), sum(v) / len(v) / 1e3, sum(v) / 1e6))


if __name__ == "__main__":
    mode, path = sys.argv[1], sys.argv[2]
    if mode == "stats":
        stats(path)
    elif mode == "trace":
        trace(path)
    elif mode == "markers":
        markers(path)
    else:
        counter(path, float(sys.argv[3]) if len(sys.argv) > 3 else None)
