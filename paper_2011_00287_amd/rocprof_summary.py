"""Summarise rocprofv3 output databases as text.

python -m paper_2011_00287_amd.rocprof_summary trace DB
    per-kernel call count, total and average duration (kernel trace)
python -m paper_2011_00287_amd.rocprof_summary counters DB [DB ...]
    per-kernel average of every collected counter (one --pmc run per DB)
python -m paper_2011_00287_amd.rocprof_summary traffic KERNEL ALGO_BYTES TRACE_DB FETCH_DB WRITE_DB
        CAL_FETCH_DB CAL_WRITE_DB CAL_BYTES OUT_JSON [--workload W --precision P]
    HBM bytes per launch of KERNEL: FETCH_SIZE and WRITE_SIZE (KiB per dispatch)
    scaled by what the same counters read on a copy kernel that reads and
    writes CAL_BYTES each, beside its algorithmic bytes and trace duration,
    stamped with the hash of the step's sources (the benchmark reports the
    traffic only while the sources still hash to it)
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


def _avg(db, kernel, counter=None):
    con = sqlite3.connect(db)
    if counter is None:
        rows = con.execute("select name, total_calls, average from top_kernels").fetchall()
        for name, calls, avg in rows:
            if name.split("(")[0].split("<")[0].split("::")[-1].strip() == kernel:
                return avg, calls
        raise KeyError(kernel)
    rows = con.execute("select kernel_name, avg(value) from counters_collection where counter_name = ? "
                       "group by kernel_name", (counter,)).fetchall()
    for name, v in rows:
        if name.split("(")[0].split("<")[0].split("::")[-1].strip() == kernel:
            return v
    raise KeyError((kernel, counter))


def _largest(db, counter):
    con = sqlite3.connect(db)
    return con.execute("select max(v) from (select avg(value) as v from counters_collection where counter_name = ? "
                       "group by kernel_name)", (counter,)).fetchone()[0]


def traffic(argv):
    import argparse
    import json
    from .build import kernel_source_hash
    ap = argparse.ArgumentParser()
    for a in ("kernel", "algo_bytes", "trace", "fetch", "write", "cal_fetch", "cal_write", "cal_bytes", "out"):
        ap.add_argument(a)
    ap.add_argument("--workload", default="droplet128")
    ap.add_argument("--precision", default="fp32")
    a = ap.parse_args(argv)
    cal = float(a.cal_bytes)
    fetch_scale = cal / (_largest(a.cal_fetch, "FETCH_SIZE") * 1024)
    write_scale = cal / (_largest(a.cal_write, "WRITE_SIZE") * 1024)
    fk = _avg(a.fetch, a.kernel, "FETCH_SIZE")
    wk = _avg(a.write, a.kernel, "WRITE_SIZE")
    us, calls = _avg(a.trace, a.kernel)
    rd, wr = fk * 1024 * fetch_scale, wk * 1024 * write_scale
    out = {"kernel": a.kernel, "workload": a.workload, "precision": a.precision, "source_hash": kernel_source_hash(),
           "fetch_size_kib": fk, "write_size_kib": wk, "fetch_scale": fetch_scale, "write_scale": write_scale,
           "hbm_bytes_per_launch": rd + wr, "hbm_read_bytes": rd, "hbm_write_bytes": wr,
           "algorithmic_bytes_per_launch": int(a.algo_bytes), "trace_average_us": us, "trace_calls": calls}
    with open(a.out, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out))


if __name__ == "__main__":
    if sys.argv[1] == "trace":
        trace(sys.argv[2])
    elif sys.argv[1] == "traffic":
        traffic(sys.argv[2:])
    else:
        counters(sys.argv[2:])
