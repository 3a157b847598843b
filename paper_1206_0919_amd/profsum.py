"""Summaries of rocprofv3 output (kernel statistics and counter runs).

    python -m paper_1206_0919_amd.profsum stats DIR      # --kernel-trace --stats
    python -m paper_1206_0919_amd.profsum pmc DIR [COUNTER...]   # --pmc runs
    python -m paper_1206_0919_amd.profsum traffic FETCH_DIR WRITE_DIR WORKLOAD \
        FETCH_SCALE WRITE_SCALE OUT_DIR DECOMPOSITION

Prints a markdown table: per kernel, calls, average duration, and for
counter runs the average counter value per dispatch.
"""
import csv
import re
import glob
import os
import sys
from collections import defaultdict


def _find(d, pattern):
    return sorted(glob.glob(os.path.join(d, "**", pattern), recursive=True))


def short(name):
    """Readable kernel name: sweep_x / sweep_y / sweep_z plus the precision.
    Accepts demangled ("void shasta::sweep_march<double, 1, 0, false>(...)")
    and mangled ("_ZN6shasta11sweep_marchIdLi1ELi0ELb0EE...") names."""
    m = re.search(r"sweep_march<(\w+), (\d)", name) or \
        re.search(r"sweep_marchI([df])Li(\d)E", name)
    if m:
        prec = "f32" if m.group(1) in ("float", "f") else "f64"
        return f"sweep_{'xyz'[int(m.group(2))]}<{prec}>"
    m = re.search(r"sweep_x<(\w+)", name) or re.search(r"sweep_xI([df])", name)
    if m:
        return "sweep_x<" + ("f32" if m.group(1) in ("float", "f") else "f64") + ">"
    for key in ("finalize_step", "stream_copy", "prim_to_cons", "read_out", "sum_fields",
                "combine_sums", "zero_doubles", "cons_in"):
        if key in name:
            return key
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


def per_dispatch(d, counter):
    """Average value of one counter per dispatch, per kernel."""
    files = _find(d, "*counter_collection.csv")
    acc = defaultdict(lambda: defaultdict(float))
    for f in files:
        for r in csv.DictReader(open(f)):
            if r.get("Counter_Name") != counter:
                continue
            name = short(r.get("Kernel_Name", "?"))
            acc[name][r.get("Dispatch_Id", "0")] += float(r["Counter_Value"])
    return {k: sum(v.values()) / len(v) for k, v in acc.items()}


def axis_key(decomposition, axis):
    """The part of a decomposition ('p0,p1,pers/...') that sets a sweep's
    HBM bytes: nothing for x (its windows are fixed by the grid), segment
    length and lanes for y and z (not the launch mode)."""
    if axis == 0:
        return ""
    return ",".join(decomposition.split("/")[axis].split(",")[:2])


def traffic(fetch_dir, write_dir, workload, fetch_scale, write_scale, out_dir, decomposition):
    """Add to profiles/traffic_<kernel>_<workload>.json the HBM bytes per
    launch = fetch_scale * FETCH_SIZE + write_scale * WRITE_SIZE (KiB) of one
    decomposition, next to the entries of other decompositions measured on
    the same kernel code (a file of other code is started afresh)."""
    import json
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    from bench import kernel_source_hash
    fe = per_dispatch(fetch_dir, "FETCH_SIZE")
    wr = per_dispatch(write_dir, "WRITE_SIZE")
    code = kernel_source_hash()
    for k in fe:
        if not k.startswith("sweep") or k not in wr:
            continue
        base = k.split("<")[0]
        axis = "xyz".index(base[-1])
        path = os.path.join(out_dir, f"traffic_{base}_{workload}.json")
        rec = {"kernel": k, "workload": workload, "source_hash": code,
               "fetch_scale": fetch_scale, "write_scale": write_scale, "entries": []}
        if os.path.exists(path):
            with open(path) as fh:
                old = json.load(fh)
            if old.get("source_hash") == code and "entries" in old:
                rec["entries"] = old["entries"]
        key = axis_key(decomposition, axis)
        rec["entries"] = [e for e in rec["entries"]
                          if axis_key(e["decomposition"], axis) != key]
        entry = {"decomposition": decomposition, "fetch_KiB": fe[k], "write_KiB": wr[k],
                 "bytes_per_launch": 1024 * (fetch_scale * fe[k] + write_scale * wr[k])}
        rec["entries"].append(entry)
        rec["entries"].sort(key=lambda e: e["decomposition"])
        with open(path, "w") as fh:
            json.dump(rec, fh, indent=1)
        print(path, decomposition, entry["bytes_per_launch"])


if __name__ == "__main__":
    mode = sys.argv[1]
    if mode == "stats":
        stats(sys.argv[2])
    elif mode == "traffic":
        # traffic FETCH_DIR WRITE_DIR WORKLOAD FETCH_SCALE WRITE_SCALE OUT_DIR DECOMPOSITION
        traffic(sys.argv[2], sys.argv[3], sys.argv[4], float(sys.argv[5]),
                float(sys.argv[6]), sys.argv[7], sys.argv[8])
    else:
        pmc(sys.argv[2], sys.argv[3:] or None)
