"""Summaries of rocprofv3 output for the step kernel (used to write profiles/).

    python -m paper_2605_25282_amd.rocprof_summary stats TRACE_kernel_stats.csv
    python -m paper_2605_25282_amd.rocprof_summary traffic FETCH_results.db WRITE_results.db KERNEL_SUBSTRING
    python -m paper_2605_25282_amd.rocprof_summary record FETCH_results.db WRITE_results.db KERNEL_SUBSTRING \
        PRECISION NODE_UPDATES_PER_LAUNCH WORKLOAD_TEXT SUMMARY_MD OUT.json

`stats` prints the kernel-statistics table of a `rocprofv3 --kernel-trace --stats
--output-format csv` run.  `traffic` reads the databases of two `rocprofv3 --pmc
FETCH_SIZE` / `--pmc WRITE_SIZE` runs of the same command, calibrates each
counter by what it reads for the plain 2 GiB device copy the profiled command
ends with (torch's copy kernel: 2 GiB read and 2 GiB written), and prints the
HBM bytes per dispatch of the kernels whose name contains KERNEL_SUBSTRING
(median over dispatches) as JSON.  `record` writes the same figures as the
traffic record the benchmark reads (with the algorithmic bytes of the given node
updates per launch and the hash of the step kernel's current sources, so the
record is ignored once the kernel changes).
"""
from __future__ import annotations

import csv
import hashlib
import json
import os
import sqlite3
import statistics
import sys

COPY_BYTES = 1 << 31  # the calibration copy: 2^28 doubles
CSRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")
STEP_KERNEL_SOURCES = ("vlbm_step_march.hip", "vlbm_device.h")
# algorithmic bytes per node update: 20 values read + 20 written; the mixed
# variant stores the populations' rho, rho v in FP32
BYTES_PER_LUP = {"fp64": 320.0, "mixed": 224.0}


def kernel_source_hash() -> str:
    """Hash of the step kernel's sources: a committed traffic measurement is
    reported only while the kernel it was taken on is unchanged."""
    h = hashlib.sha256()
    for f in STEP_KERNEL_SOURCES:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def kernel_stats(path: str) -> list[dict]:
    """Rows of a rocprofv3 kernel_stats.csv (name, calls, total/avg ns, percent)."""
    out = []
    with open(path, newline="") as f:
        for row in csv.DictReader(f):
            out.append({"name": row["Name"], "calls": int(row["Calls"]),
                        "total_ms": float(row["TotalDurationNs"]) / 1e6,
                        "avg_us": float(row["AverageNs"]) / 1e3,
                        "percent": float(row["Percentage"])})
    return out


def _per_dispatch(db: str, counter: str) -> list[tuple[str, float]]:
    """(kernel name, counter value summed over its instances) for every dispatch, in order."""
    c = sqlite3.connect(db)
    rows = c.execute("select dispatch_id, kernel_name, sum(value) from counters_collection "
                     "where counter_name = ? group by dispatch_id, kernel_name order by dispatch_id",
                     (counter,)).fetchall()
    c.close()
    return [(k, float(v)) for _, k, v in rows]


def traffic(fetch_db: str, write_db: str, kernel: str) -> dict:
    """Calibrated HBM bytes per dispatch of `kernel` from FETCH_SIZE / WRITE_SIZE (KiB)."""
    res = {}
    for name, db, counter in (("fetch", fetch_db, "FETCH_SIZE"), ("write", write_db, "WRITE_SIZE")):
        rows = _per_dispatch(db, counter)
        copies = [v for k, v in rows if "copy" in k.lower() or "elementwise" in k.lower()]
        if not copies:
            raise RuntimeError(f"{db}: no calibration copy dispatch found")
        # the calibration copy is the last copy-like dispatch of the run
        scale = COPY_BYTES / (copies[-1] * 1024.0)
        vals = [v * 1024.0 * scale for k, v in rows if kernel in k]
        res[name] = {"raw_kib_per_dispatch": [round(v / 1024.0 / scale, 1) for v in vals],
                     "copy_raw_kib": copies[-1], "scale": round(scale, 4),
                     "median_bytes": statistics.median(vals)}
    res["bytes_per_launch"] = res["fetch"]["median_bytes"] + res["write"]["median_bytes"]
    return res


def record(fetch_db: str, write_db: str, kernel: str, precision: str, node_updates: float, workload: str,
           source: str) -> dict:
    """Traffic record of one workload: calibrated bytes per launch, the
    algorithmic bytes of its node updates and the step kernel's source hash."""
    t = traffic(fetch_db, write_db, kernel)
    return {"bytes_per_launch": t["bytes_per_launch"],
            "fetch_bytes": t["fetch"]["median_bytes"], "write_bytes": t["write"]["median_bytes"],
            "node_updates_per_launch": node_updates,
            "algorithmic_bytes_per_launch": BYTES_PER_LUP[precision] * node_updates,
            "kernel": kernel, "workload": workload, "kernel_source_hash": kernel_source_hash(),
            "source": source, "hashed_sources": list(STEP_KERNEL_SOURCES)}


def main(argv: list[str]) -> int:
    if len(argv) >= 2 and argv[0] == "stats":
        print("| kernel | calls | total ms | avg us | % |\n|---|---|---|---|---|")
        for r in kernel_stats(argv[1]):
            print(f"| `{r['name'][:90]}` | {r['calls']} | {r['total_ms']:.2f} | {r['avg_us']:.1f} | "
                  f"{r['percent']:.2f} |")
        return 0
    if len(argv) == 4 and argv[0] == "traffic":
        print(json.dumps(traffic(argv[1], argv[2], argv[3]), indent=1))
        return 0
    if len(argv) == 9 and argv[0] == "record":
        rec = record(argv[1], argv[2], argv[3], argv[4], float(argv[5]), argv[6], argv[7])
        with open(argv[8], "w") as f:
            json.dump(rec, f, indent=1)
            f.write("\n")
        print(json.dumps(rec, indent=1))
        return 0
    print(__doc__)
    return 2


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
