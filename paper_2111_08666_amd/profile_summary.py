"""Summarise rocprofv3 output (its SQLite results database, or kernel-stats
and counter CSVs) into a short text table: per kernel, the dispatch count,
mean duration and the mean of each collected counter per dispatch.

    python -m paper_2111_08666_amd.profile_summary <rocprofv3 output dir>...
"""
import csv
import glob
import os
import sqlite3
import sys
from collections import defaultdict


def short(name, n=60):
    name = name.replace("void lbm::", "").split("(")[0]
    return name if len(name) <= n else name[:n]


def summarize_db(f, root):
    out = [f"# rocprofv3 database: {os.path.relpath(f, root)}"]
    db = sqlite3.connect(f)
    cur = db.cursor()
    rows = cur.execute("select name, count(*), avg(duration), sum(duration) from kernels "
                       "group by name order by sum(duration) desc").fetchall()
    if rows:
        total = sum(r[3] for r in rows)
        out.append(f"{'kernel':62s} {'calls':>6s} {'mean_us':>10s} {'total_ms':>10s} {'pct':>6s}")
        for name, n, avg, tot in rows:
            out.append(f"{short(name):62s} {n:6d} {avg / 1e3:10.2f} {tot / 1e6:10.3f} {100 * tot / total:6.2f}")
    try:
        ev = cur.execute("select name, dispatch_id, counter_name, sum(counter_value) from pmc_events "
                         "group by name, dispatch_id, counter_name").fetchall()
    except sqlite3.Error:
        ev = []
    acc = defaultdict(lambda: defaultdict(list))
    for name, _, cname, val in ev:
        acc[short(name)][cname].append(val)
    for k, cs in acc.items():
        vals = ", ".join(f"{c}={sum(v) / len(v):.5g}" for c, v in sorted(cs.items()))
        n = max(len(v) for v in cs.values())
        out.append(f"{k:62s} dispatches={n} {vals}")
    return out


def summarize(path):
    out = []
    for f in sorted(glob.glob(os.path.join(path, "**", "*.db"), recursive=True)):
        out += summarize_db(f, path)
    for f in sorted(glob.glob(os.path.join(path, "**", "*kernel_stats.csv"), recursive=True)):
        out.append(f"# kernel stats: {os.path.relpath(f, path)}")
        with open(f) as fh:
            rows = list(csv.DictReader(fh))
        out.append(f"{'kernel':62s} {'calls':>6s} {'mean_us':>10s} {'total_ms':>10s} {'pct':>6s}")
        for r in rows:
            out.append(f"{short(r['Name']):62s} {int(r['Calls']):6d} {float(r['AverageNs']) / 1e3:10.2f} "
                       f"{float(r['TotalDurationNs']) / 1e6:10.3f} {float(r['Percentage']):6.2f}")
    for f in sorted(glob.glob(os.path.join(path, "**", "*counter_collection.csv"), recursive=True)):
        out.append(f"# counters: {os.path.relpath(f, path)}")
        acc = defaultdict(lambda: defaultdict(list))
        with open(f) as fh:
            for r in csv.DictReader(fh):
                acc[short(r["Kernel_Name"])][r["Counter_Name"]].append(float(r["Counter_Value"]))
        for k, cs in acc.items():
            vals = ", ".join(f"{c}={sum(v) / len(v):.4g}" for c, v in sorted(cs.items()))
            n = max(len(v) for v in cs.values())
            out.append(f"{k:62s} dispatches={n} {vals}")
    return "\n".join(out)


if __name__ == "__main__":
    for p in sys.argv[1:]:
        print(summarize(p))
