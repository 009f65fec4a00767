"""Summarise rocprofv3 output databases as text.

python -m paper_2011_00287_amd.rocprof_summary trace DB
    per-kernel call count, total and average duration (kernel trace)
python -m paper_2011_00287_amd.rocprof_summary counters DB [DB ...]
    per-kernel average of every collected counter (one --pmc run per DB)
"""
from __future__ import annotations

import sqlite3
import sys


def trace(db):
    con = sqlite3.connect(db)
    rows = con.execute("select name, total_calls, total_duration, average, percentage from top_kernels").fetchall()
    print("| kernel | calls | total (us) | average (us) | % |")
    print("|---|---|---|---|---|")
    for name, calls, tot, avg, pct in rows:  # durations are reported in microseconds
        print(f"| {name.split('(')[0]} | {calls} | {tot:.1f} | {avg:.3f} | {pct:.1f} |")


def counters(dbs):
    print("| kernel | counter | average per dispatch | dispatches |")
    print("|---|---|---|---|")
    for db in dbs:
        con = sqlite3.connect(db)
        rows = con.execute("select kernel_name, counter_name, avg(value), count(*) from counters_collection "
                           "group by kernel_name, counter_name order by kernel_name").fetchall()
        for k, c, v, n in rows:
            print(f"| {k.split('(')[0]} | {c} | {v:.1f} | {n} |")


if __name__ == "__main__":
    if sys.argv[1] == "trace":
        trace(sys.argv[2])
    else:
        counters(sys.argv[2:])
