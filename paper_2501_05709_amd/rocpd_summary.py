"""Summarise rocprofv3 databases (rocpd SQLite) per kernel.

    python -m paper_2501_05709_amd.rocpd_summary DB [DB ...] [--match SUBSTR]

Prints, per kernel name and per counter, the number of dispatches and the
mean value per dispatch (counters) or the mean duration (kernel traces), as a
markdown table.  Only the standard library is used.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sqlite3
from collections import defaultdict


def counters(db):
    con = sqlite3.connect(db)
    rows = con.execute("select kernel_name, counter_name, value, duration, grid_size from counters_collection")
    agg = defaultdict(lambda: [0, 0.0, 0.0, 0])
    for name, cname, value, dur, grid in rows:
        a = agg[(name, cname)]
        a[0] += 1
        a[1] += float(value)
        a[2] += float(dur or 0)
        a[3] = grid
    return agg


def kernels(db):
    con = sqlite3.connect(db)
    rows = con.execute("select name, duration from kernels")
    agg = defaultdict(lambda: [0, 0.0])
    for name, dur in rows:
        a = agg[name]
        a[0] += 1
        a[1] += float(dur)
    return agg


def traffic_entry(fetch_db, write_db, kernel, copy_bytes):
    """HBM bytes per launch of the kernels whose names match the regular expression
    `kernel` (all their dispatches together: the RK-stage instances of one kernel, say),
    from FETCH_SIZE and WRITE_SIZE runs, each scaled by what the same counter reads for
    the calibration copy (copy_bytes read and written), the first copy of the run."""
    pat = re.compile(kernel)

    def per_kernel(db, counter):
        agg = counters(db)
        k = [v for (name, c), v in agg.items() if c == counter and pat.search(name)]
        if not k:
            raise SystemExit(f"no dispatch of a kernel matching {kernel!r} with {counter} in {db}")
        con = sqlite3.connect(db)
        # the calibration copy is the first device copy of the run (bench.py
        # --calibrate-copy copies copy_bytes before anything else); larger copies may
        # follow (a batch's FP64 state saved by the autotuner)
        first = con.execute(
            "select value from counters_collection where counter_name = ? and kernel_name like '%copyBuffer%' "
            "order by dispatch_id limit 1", (counter,)).fetchone()
        return sum(v[1] for v in k) / sum(v[0] for v in k), float(first[0])
    f_k, f_copy = per_kernel(fetch_db, "FETCH_SIZE")
    w_k, w_copy = per_kernel(write_db, "WRITE_SIZE")
    f_scale = copy_bytes / (f_copy * 1024.0)
    w_scale = copy_bytes / (w_copy * 1024.0)
    return {"fetch_kib": round(f_k, 1), "write_kib": round(w_k, 1),
            "copy_fetch_kib": round(f_copy, 1), "copy_write_kib": round(w_copy, 1),
            "fetch_scale": round(f_scale, 4), "write_scale": round(w_scale, 4),
            "hbm_bytes_per_launch": round(f_k * 1024.0 * f_scale + w_k * 1024.0 * w_scale)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("db", nargs="+")
    ap.add_argument("--match", default="")
    ap.add_argument("--traffic", nargs=4, metavar=("WORKLOAD", "KERNEL_REGEX", "FETCH_DB", "WRITE_DB"),
                    help="write the counter traffic of the kernels matching KERNEL_REGEX into "
                         "profiles/counters.json, keyed by the name before the template arguments")
    ap.add_argument("--copy-bytes", type=float, default=2.0 ** 30)
    args = ap.parse_args()
    if args.traffic:
        workload, kernel, fdb, wdb = args.traffic
        root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
        src = open(os.path.join(root, "paper_2501_05709_amd", "csrc", "fr_kernels.hip"), "rb").read()
        entry = traffic_entry(fdb, wdb, kernel, args.copy_bytes)
        entry["source_sha256"] = hashlib.sha256(src).hexdigest()
        entry["kernel_match"] = kernel
        path = os.path.join(root, "profiles", "counters.json")
        data = json.load(open(path)) if os.path.exists(path) else {}
        data.setdefault(workload, {})[re.split(r"[<\\]", kernel)[0]] = entry
        json.dump(data, open(path, "w"), indent=1, sort_keys=True)
        print(json.dumps(entry))
        return
    print("| kernel | counter | dispatches | mean per dispatch | grid |")
    print("|---|---|---|---|---|")
    for db in args.db:
        try:
            agg = counters(db)
        except sqlite3.OperationalError:
            agg = {}
        for (name, cname), (n, tot, dur, grid) in sorted(agg.items()):
            if args.match and args.match not in name:
                continue
            print(f"| {name} | {cname} | {n} | {tot / n:.1f} | {grid} |")
        if not agg:
            for name, (n, tot) in sorted(kernels(db).items(), key=lambda kv: -kv[1][1]):
                if args.match and args.match not in name:
                    continue
                print(f"| {name} | duration_ns | {n} | {tot / n:.0f} | |")


if __name__ == "__main__":
    main()
