"""Summaries of rocprofv3 output (kernel statistics and counter runs).

    python -m paper_1206_0919_amd.profsum stats DIR      # --kernel-trace --stats
    python -m paper_1206_0919_amd.profsum pmc DIR [COUNTER...]   # --pmc runs

Prints a markdown table: per kernel, calls, average duration, and for
counter runs the average counter value per dispatch.
"""
import csv
import glob
import os
import sys
from collections import defaultdict


def _find(d, pattern):
    return sorted(glob.glob(os.path.join(d, "**", pattern), recursive=True))


def short(name):
    for key in ("sweep_x", "sweep_march", "finalize_step", "stream_copy", "prim_to_cons",
                "read_out", "sum_fields", "combine_sums", "zero_doubles", "cons_in"):
        if key in name:
            tail = name.split(key, 1)[1]
            args = tail[tail.find("I") + 1:tail.find("EE")] if "I" in tail[:3] else ""
            return key + (f"<{args}>" if args else "")
    return name[:60]


def stats(d):
    files = _find(d, "*kernel_stats.csv")
    if not files:
        print(f"no kernel_stats.csv under {d}")
        return
    print("| kernel | calls | avg us | min us | max us | total ms |")
    print("|---|---:|---:|---:|---:|---:|")
    for f in files:
        for r in csv.DictReader(open(f)):
            calls = int(r["Calls"])
            print(f"| {short(r['Name'])} | {calls} | {float(r['AverageNs'])/1e3:.1f} | "
                  f"{float(r['MinNs'])/1e3:.1f} | {float(r['MaxNs'])/1e3:.1f} | "
                  f"{float(r['TotalDurationNs'])/1e6:.3f} |")


def pmc(d, counters=None):
    files = _find(d, "*counter_collection.csv")
    if not files:
        print(f"no counter_collection.csv under {d}")
        return
    acc = defaultdict(lambda: defaultdict(list))
    for f in files:
        for r in csv.DictReader(open(f)):
            name = short(r.get("Kernel_Name", r.get("Kernel-Name", "?")))
            cname = r.get("Counter_Name", r.get("Counter-Name"))
            if counters and cname not in counters:
                continue
            key = r.get("Dispatch_Id", r.get("Correlation_Id", "0"))
            acc[name][cname].append((key, float(r["Counter_Value"])))
    print("| kernel | counter | dispatches | avg per dispatch |")
    print("|---|---|---:|---:|")
    for name, cs in acc.items():
        for cname, vals in cs.items():
            per = defaultdict(float)
            for k, v in vals:
                per[k] += v
            avg = sum(per.values()) / len(per)
            print(f"| {name} | {cname} | {len(per)} | {avg:.6g} |")


if __name__ == "__main__":
    mode, d = sys.argv[1], sys.argv[2]
    if mode == "stats":
        stats(d)
    else:
        pmc(d, sys.argv[3:] or None)
