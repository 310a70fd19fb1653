"""Summarise rocprofv3 output (its SQLite results database, or kernel-stats
and counter CSVs) into a short text table: per kernel, the dispatch count,
mean duration and the mean of each collected counter per dispatch.

    python -m paper_2111_08666_amd.profile_summary <rocprofv3 output dir>...
"""
import csv
import glob
import os
import sqlite3
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


def _dispatch_values(path, counter):
    """{kernel name: [per-dispatch value]} for one counter over a run's databases."""
    vals = defaultdict(list)
    for f in sorted(glob.glob(os.path.join(path, "**", "*.db"), recursive=True)):
        cur = sqlite3.connect(f).cursor()
        for name, _, v in cur.execute("select name, dispatch_id, sum(counter_value) from pmc_events "
                                      "where counter_name = ? group by name, dispatch_id", (counter,)):
            vals[name].append(v)
    return vals


def traffic(fetch_dir, write_dir, kernel, copy_mib):
    """HBM bytes per launch of `kernel` (substring of the full name) from a
    FETCH_SIZE run and a WRITE_SIZE run (KiB per dispatch), each scaled by
    the factor that makes the largest copy dispatches of the same run read
    and write `copy_mib` MiB."""
    out = {}
    for counter, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        vals = _dispatch_values(d, counter)
        cv = sorted((v for n, vs in vals.items() if "copyBuffer" in n for v in vs), reverse=True)[:3]
        if not cv:
            raise SystemExit(f"no calibration copy in {d}")
        factor = copy_mib * 1024.0 / (sum(cv) / len(cv))
        kib, disp = 0.0, []
        for part in kernel.split("+"):   # a step of several kernels: sum their means
            kv = [v for n, vs in vals.items() if part.strip() in n for v in vs]
            if not kv:
                raise SystemExit(f"no dispatches of {part!r} in {d}")
            kib += sum(kv) / len(kv)
            disp.append(len(kv))
        out[counter] = {"kib_per_launch": kib, "dispatches": disp, "scale": factor,
                        "bytes_per_launch": kib * 1024.0 * factor}
    out["bytes_per_launch"] = out["FETCH_SIZE"]["bytes_per_launch"] + out["WRITE_SIZE"]["bytes_per_launch"]
    return out


def main():
    import argparse
    import json
    ap = argparse.ArgumentParser()
    ap.add_argument("dirs", nargs="*")
    ap.add_argument("--traffic", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"))
    ap.add_argument("--kernel", help="substring of the profiled kernel's full name ('a+b+c': a step of "
                                     "several kernels)")
    ap.add_argument("--name", help="kernel name as the solver reports it")
    ap.add_argument("--workload")
    ap.add_argument("--copy-mib", type=int, default=1024)
    ap.add_argument("--out", default="")
    a = ap.parse_args()
    for p in a.dirs:
        print(summarize(p))
    if a.traffic:
        from paper_2111_08666_amd.build import kernel_source_hash
        rec = traffic(a.traffic[0], a.traffic[1], a.kernel, a.copy_mib)
        rec["source_hash"] = kernel_source_hash()
        print(json.dumps({f"{a.name}|{a.workload}": rec}, indent=1))
        if a.out:
            data = {}
            if os.path.exists(a.out):
                with open(a.out) as f:
                    data = json.load(f)
            data[f"{a.name}|{a.workload}"] = rec
            with open(a.out, "w") as f:
                json.dump(data, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main()
