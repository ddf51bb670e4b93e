"""Kernel summary (calls, total/avg/min/max us, share) of a rocprofv3 kernel trace.

Reads a rocpd database (run_results.db), a kernel-trace CSV
(run_kernel_trace.csv) or the per-kernel statistics CSV that --stats writes
(run_kernel_stats.csv: calls, total, min and max per kernel, no dispatches). Persistent batched kernels are listed as
k_persist<Desc> (the profiler prints them mangled). The last block gives the
product kernel classes (launch count and average duration), the figures the
benchmark's launch-timing hooks report for the same classes.

usage: python -m paper_2506_04840_amd.rocpd_summary <run_results.db | run_kernel_trace.csv | run_kernel_stats.csv> [top_n]
"""
import collections
import csv
import re
import sqlite3
import sys

from .pmc_traffic import CLASSES


def _rows(path):
    """(name, duration_ns) of every kernel dispatch."""
    if path.endswith(".csv"):
        for r in csv.DictReader(open(path)):
            yield r["Kernel_Name"], int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
    else:
        c = sqlite3.connect(path)
        for name, dur in c.execute("select name, duration from kernels"):
            yield name, int(dur)


def _short(name):
    m = re.match(r"_ZN2tk9k_persistINS_\d+(\w+?)E", name)
    if m:
        inner = re.search(r"_ZNS_\d+(b_\w+?)(?:ILi(\d+)E)?E", name)
        body = inner.group(1) + ("<%s>" % inner.group(2) if inner and inner.group(2) else "") if inner else "?"
        return "k_persist<%s, %s>" % (m.group(1), body)
    return name.split("(")[0]


def _stats(path):
    """(name, calls, total_ns, min_ns, max_ns) per kernel: aggregated from the
    dispatches of a trace or database, or read from a --stats CSV."""
    if path.endswith("kernel_stats.csv"):
        for r in csv.DictReader(open(path)):
            yield r["Name"], int(r["Calls"]), int(r["TotalDurationNs"]), int(r["MinNs"]), int(r["MaxNs"])
        return
    per = collections.defaultdict(list)
    for name, dur in _rows(path):
        per[name].append(dur)
    for name, v in per.items():
        yield name, len(v), sum(v), min(v), max(v)


def main():
    path = sys.argv[1]
    top = int(sys.argv[2]) if len(sys.argv) > 2 else 30
    agg = {}  # short name -> [calls, total, min, max]
    cls = collections.defaultdict(lambda: [0, 0])
    for name, calls, tot, lo, hi in _stats(path):
        a = agg.setdefault(_short(name), [0, 0, lo, hi])
        a[0] += calls
        a[1] += tot
        a[2] = min(a[2], lo)
        a[3] = max(a[3], hi)
        for k, rx in CLASSES.items():
            if re.search(rx, name):
                cls[k][0] += calls
                cls[k][1] += tot
    total = sum(v[1] for v in agg.values())
    print("%-70s %7s %12s %10s %10s %10s %6s" % ("kernel", "calls", "total_us", "avg_us", "min_us", "max_us", "pct"))
    for name, (n, tot, lo, hi) in sorted(agg.items(), key=lambda kv: -kv[1][1])[:top]:
        print("%-70s %7d %12.1f %10.2f %10.2f %10.2f %6.2f" % (name[:70], n, tot / 1e3, tot / n / 1e3, lo / 1e3,
                                                              hi / 1e3, 100.0 * tot / total))
    print()
    print("%-24s %7s %12s %10s" % ("kernel class", "calls", "total_us", "avg_us"))
    for k, (n, tot) in cls.items():
        print("%-24s %7d %12.1f %10.2f" % (k, n, tot / 1e3, tot / n / 1e3))


if __name__ == "__main__":
    main()
