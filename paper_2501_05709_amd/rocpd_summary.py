"""Summarise rocprofv3 databases (rocpd SQLite) per kernel.

    python -m paper_2501_05709_amd.rocpd_summary DB [DB ...] [--match SUBSTR]

Prints, per kernel name and per counter, the number of dispatches and the
mean value per dispatch (counters) or the mean duration (kernel traces), as a
markdown table.  Only the standard library is used.
"""
from __future__ import annotations

import argparse
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("db", nargs="+")
    ap.add_argument("--match", default="")
    args = ap.parse_args()
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
