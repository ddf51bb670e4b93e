"""HBM traffic per launch of a kernel class from rocprofv3 counter runs.

Inputs are the counter-collection CSVs of four runs, each with one counter:
FETCH_SIZE and WRITE_SIZE (KiB per dispatch) of the benchmark, and the same
two counters for a plain device copy of a known number of bytes. The copy
calibrates each counter (reported KiB * 1024 / bytes moved); the kernel's
counts are divided by that factor.

usage: python -m paper_2506_04840_amd.pmc_traffic --fetch F.csv --write W.csv \
           --copy-fetch CF.csv --copy-write CW.csv --copy-bytes N \
           --kernel colreduce --workload hilbert3_400 [--json out.json]
"""
from __future__ import annotations

import argparse
import collections
import csv
import hashlib
import json
import os
import re

CLASSES = {
    "colreduce": r"tk::k_cr_(lds|cols|split)<",
    "rowcontract": r"tk::k_rc_(rows|cols|split)<",
    "powerstep": r"tk::k_power_(fused|split)<",
    # persistent batched kernels: the profiler may print them mangled
    "batched_colreduce": r"k_persist<tk::BCr(Split|Lds|Cols),|k_persistINS_\d+BCr(Split|Lds|Cols)E",
    "batched_rowcontract": r"k_persist<tk::BRc(Split|Rows|Cols),|k_persistINS_\d+BRc(Split|Rows|Cols)E",
}
COPY = r"__amd_rocclr_copyBuffer"
CSRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")


SOURCES = ("ttm.hip", "common.hpp", "internal.hpp", "api.cpp")


def source_digest() -> str:
    """sha256 over the sources that shape the product launches the counters
    describe (kernels, persistent wrapper, launch and split policies)."""
    h = hashlib.sha256()
    for name in SOURCES:
        with open(os.path.join(CSRC, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def _rows(path: str, pattern: str):
    rx = re.compile(pattern)
    return [r for r in csv.DictReader(open(path)) if rx.search(r["Kernel_Name"])]


def _copy_factor(path: str, nbytes: int) -> float:
    vals = [float(r["Counter_Value"]) for r in _rows(path, COPY)]
    if not vals:
        raise SystemExit("no copy kernel in %s" % path)
    return sum(vals) / len(vals) * 1024.0 / nbytes


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--fetch", required=True)
    ap.add_argument("--write", required=True)
    ap.add_argument("--copy-fetch", required=True)
    ap.add_argument("--copy-write", required=True)
    ap.add_argument("--copy-bytes", type=int, required=True)
    ap.add_argument("--kernel", default="colreduce", choices=sorted(CLASSES))
    ap.add_argument("--workload", required=True)
    ap.add_argument("--json", default=None)
    a = ap.parse_args()
    ff = _copy_factor(a.copy_fetch, a.copy_bytes)
    fw = _copy_factor(a.copy_write, a.copy_bytes)
    fetch = _rows(a.fetch, CLASSES[a.kernel])
    write = _rows(a.write, CLASSES[a.kernel])
    if not fetch or len(fetch) != len(write):
        raise SystemExit("launch counts differ or are zero: %d fetch, %d write" % (len(fetch), len(write)))
    per = collections.defaultdict(lambda: [0, 0.0, 0.0])
    for r in fetch:
        k = (r["Kernel_Name"].split("(")[0], r["Grid_Size"])
        per[k][0] += 1
        per[k][1] += float(r["Counter_Value"]) * 1024.0 / ff
    for r in write:
        k = (r["Kernel_Name"].split("(")[0], r["Grid_Size"])
        per[k][2] += float(r["Counter_Value"]) * 1024.0 / fw
    launches = len(fetch)
    total = sum(v[1] + v[2] for v in per.values())
    print("kernel class %s, workload %s: %d launches" % (a.kernel, a.workload, launches))
    print("copy calibration: FETCH_SIZE reads %.4f, WRITE_SIZE reads %.4f of the bytes moved" % (ff, fw))
    print("%-48s %9s %6s %14s %14s" % ("kernel", "grid", "calls", "read MB/call", "write MB/call"))
    for (name, grid), (n, rd, wr) in sorted(per.items(), key=lambda kv: -kv[1][1]):
        print("%-48s %9s %6d %14.2f %14.2f" % (name[:48], grid, n, rd / n / 1e6, wr / n / 1e6))
    print("HBM traffic per launch (class average): %.1f MB" % (total / launches / 1e6))
    if a.json:
        with open(a.json, "w") as f:
            json.dump({"kernel": a.kernel, "workload": a.workload, "launches": launches,
                       "traffic_bytes_per_launch": total / launches, "fetch_factor": ff, "write_factor": fw,
                       "source_sha256": source_digest()}, f, indent=1)
            f.write("\n")


if __name__ == "__main__":
    main()
