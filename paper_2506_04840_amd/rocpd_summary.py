"""Print a kernel summary (calls, total/avg/min/max us, share) from a rocprofv3 rocpd database.

usage: python -m paper_2506_04840_amd.rocpd_summary <run_results.db> [top_n]
"""
import sqlite3
import sys


def main():
    db = sys.argv[1]
    top = int(sys.argv[2]) if len(sys.argv) > 2 else 30
    c = sqlite3.connect(db)
    rows = list(c.execute(
        "select name, count(*), sum(duration), avg(duration), min(duration), max(duration) "
        "from kernels group by name order by sum(duration) desc"))
    total = sum(r[2] for r in rows)
    print("%-70s %7s %12s %10s %10s %10s %6s" % ("kernel", "calls", "total_us", "avg_us", "min_us", "max_us", "pct"))
    for name, n, tot, avg, mn, mx in rows[:top]:
        short = name.split("(")[0][:70]
        print("%-70s %7d %12.1f %10.2f %10.2f %10.2f %6.2f" % (short, n, tot / 1e3, avg / 1e3, mn / 1e3, mx / 1e3,
                                                              100.0 * tot / total))


if __name__ == "__main__":
    main()
