#!/usr/bin/env python3
"""Benchmark of the relativistic SHASTA time step on one MI355X.

    python bench.py [--steps K] [--warmup W] [--workload NAME] [--no-legs] [--bag400]
                    [--variants]

A step is one full time step (three directional sweeps and the step
reductions) of the whole batch, with the state resident in HBM.  After W
warm-up steps and one captured and replayed 6-step graph cycle, K steps are
timed five times; the value is the median.  Prints one JSON line with
cell-updates/s, the roofline of the dominant kernel (HIP-event timing of each
launch on the library's stream, algorithmic bytes per launch), the FP32-mixed
and batched legs of the metric (each with its throughput, roofline and field
error against the FP64 path) and the FP64 CPU oracle timed on a bounded
sample on the host cores.

Workloads (synthetic, seeded):
  hotspots200     200^3, dx 0.2 fm, dt/dx 0.4, p = e/3, 64 Gaussian hot spots,
                  FP64 (default: the configuration the metric is quoted on)
  shock256_mixed  256^3 planar shock tube, FP32 fields + FP64 recovery
  batch96         96 events, axes from {48,64,96,128}, FP32 + FP64 recovery
  bag400          400^3, dx 0.1 fm, bag-model EOS, FP32 + FP64 recovery
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
FIELD_PASSES = 2 * 5           # one read and one write of five fields per sweep


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def code_tokens(src):
    """C/C++ source without comments, whitespace runs collapsed to one space
    (string and character literals kept as written)."""
    out, i, n = [], 0, len(src)
    while i < n:
        c = src[i]
        if src.startswith("//", i):
            j = src.find("\n", i)
            i = n if j < 0 else j
        elif src.startswith("/*", i):
            j = src.find("*/", i + 2)
            i = n if j < 0 else j + 2
            out.append(" ")
        elif c in "\"'":
            j = i + 1
            while j < n and src[j] != c:
                j += 2 if src[j] == "\\" else 1
            out.append(src[i:j + 1])
            i = j + 1
        else:
            out.append(c)
            i += 1
    return " ".join("".join(out).split())


def kernel_source_hash(read=None):
    """Hash of the kernel sources as code: comments and layout do not count,
    so a counter summary stays valid across edits that change neither."""
    h = hashlib.sha256()
    for f in ("shasta_sweeps.hpp", "shasta_kernels.hip", "shasta_math.hpp",
              "shasta_internal.hpp"):
        if read is None:
            with open(os.path.join(ROOT, "paper_1206_0919_amd", "csrc", f)) as fh:
                text = fh.read()
        else:
            text = read(f)
        h.update(code_tokens(text).encode())
    return h.hexdigest()[:16]


def measured_traffic(kernel, workload, decomposition):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel code with a decomposition that gives the
    kernel's axis the same bytes; else None."""
    from paper_1206_0919_amd.profsum import axis_key
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if d.get("source_hash") != kernel_source_hash():
        return None
    axis = "xyz".index(kernel[-1])
    key = axis_key(decomposition, axis)
    for e in d.get("entries", []):
        if axis_key(e["decomposition"], axis) == key:
            return e["bytes_per_launch"]
    return None


def copy_ceiling(torch, B, mib=1024, reps=10):
    """Achievable HBM bandwidth: the library's plain copy kernel on `mib` MiB,
    timed with HIP events on the current stream (read + write bytes)."""
    n = mib << 20
    src = torch.ones(n // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    st = torch.cuda.current_stream()
    for _ in range(3):
        B.stream_copy(src, dst, n, st)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(st)
    for _ in range(reps):
        B.stream_copy(src, dst, n, st)
    b.record(st)
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    del src, dst
    return 2 * n / (ms * 1e-3) / 1e9


def pattern_floor(torch, B, dims, precision, decomposition, reps=10):
    """Average time of the y and z sweeps' memory pattern without their
    arithmetic (the library's march copy: same segment length as the
    decomposition, flattened lanes, same halo rows), timed with HIP events on
    the current stream; with the algorithmic bytes of a sweep as GB/s."""
    nx, ny, nz = dims
    ncell = nx * ny * nz
    dt = torch.float64 if precision == B.FP64 else torch.float32
    esize = 8 if precision == B.FP64 else 4
    src = torch.ones(5 * ncell, dtype=dt, device="cuda")
    dst = torch.empty_like(src)
    st = torch.cuda.current_stream()
    out = {}
    for axis, name in ((1, "sweep_y"), (2, "sweep_z")):
        seg = int(decomposition.split("/")[axis].split(",")[0]) or dims[axis]
        for _ in range(3):
            B.march_copy(src, dst, dims, ncell, axis, seg, precision, st)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(st)
        for _ in range(reps):
            B.march_copy(src, dst, dims, ncell, axis, seg, precision, st)
        b.record(st)
        torch.cuda.synchronize()
        us = 1000.0 * a.elapsed_time(b) / reps
        out[name] = {"segment": seg, "avg_us": us,
                     "GBs": ncell * FIELD_PASSES * esize / (us * 1e-6) / 1e9}
    del src, dst
    return out


def make_state(torch, B, wl, precision):
    dims = wl["dims"] if isinstance(wl["dims"], list) else [wl["dims"]]
    kind, params = wl["eos"]
    eos = (B.EOS_BAG, params) if kind == "bag" else None
    t0 = time.time()
    prims = wl["init"]()
    if not isinstance(prims, list):
        prims = [prims]
    log(f"initial state generated in {time.time() - t0:.1f}s")
    s = B.Shasta(dims, wl["dx"], precision=precision, eos=eos)
    for k, pr in enumerate(prims):
        s.write_primitive(k, *[torch.from_numpy(a) for a in pr.as_tuple()])
    cells = sum(d[0] * d[1] * d[2] for d in dims)
    return s, prims, cells


def warm_through_cycle(torch, s, dt, warmup):
    """`warmup` steps, then on to the next multiple of 6 steps and one whole
    6-step cycle: the step graph is captured and replayed before any timed
    step (the timed steps reuse it: the buffer parity is the same at every
    multiple of 6 steps)."""
    s.step(dt, warmup)
    k = s.step_index()
    s.step(dt, (-k) % 6 + 6)
    torch.cuda.synchronize()


def time_steps(torch, s, dt, steps):
    st = s.stream
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record(st)
    s.step(dt, steps)
    b.record(st)
    torch.cuda.synchronize()
    return a.elapsed_time(b)


def kernel_profile(torch, s, dt, steps):
    s.set_profiling(True)
    s.step(dt, steps)
    ms, n = s.read_profile()
    s.set_profiling(False)
    names = ("sweep_x", "sweep_y", "sweep_z", "step_reduce")
    return {names[i]: dict(ms_total=ms[i], launches=n[i],
                           avg_us=1000.0 * ms[i] / n[i] if n[i] else None)
            for i in range(4)}


def cpu_baseline(wl, prims, budget_s=20.0):
    import numpy as np
    import oracle
    kind, params = wl["eos"]
    o = oracle.Oracle(oracle.EOS_BAG, *params) if kind == "bag" else oracle.Oracle()
    cores = o.max_threads()
    pr = prims[0]
    dims = pr.e.shape[::-1]
    U = [np.ascontiguousarray(a.reshape(pr.e.shape)) for a in o.prim_to_cons(*pr.as_tuple())]
    cells = int(np.prod(dims))
    # one step first, to size the sample to the time budget
    t0 = time.perf_counter()
    o.run(U, wl["lam"], 1, k0=0)
    t1 = time.perf_counter() - t0
    n = max(1, min(50, int(budget_s / max(t1, 1e-6)) - 1))
    t0 = time.perf_counter()
    o.run(U, wl["lam"], n, k0=1)
    t = time.perf_counter() - t0
    # the same oracle on one thread, continuing from the same state (bounded
    # to about a third of the budget)
    t0 = time.perf_counter()
    o.run(U, wl["lam"], 1, k0=n + 1, nthreads=1)
    t1s = time.perf_counter() - t0
    n1 = max(0, min(10, int(budget_s / 3 / max(t1s, 1e-6)) - 1))
    if n1:
        t0 = time.perf_counter()
        o.run(U, wl["lam"], n1, k0=n + 2, nthreads=1)
        t1s = (time.perf_counter() - t0) / n1
    cpu = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            cpu = next((l.split(":", 1)[1].strip() for l in fh if l.startswith("model name")),
                       cpu)
    except OSError:
        pass
    return dict(value=cells * n / t, unit="cell-updates/s", cores=cores, kind="oracle",
                sample=f"{wl['name']} event 0 ({dims[0]}x{dims[1]}x{dims[2]}), steps 2..{n + 1} "
                       f"of the FP64 oracle, OpenMP over pencils, {cores} threads, {t:.1f}s",
                single_thread=dict(value=cells / t1s, unit="cell-updates/s",
                                   sample=f"{max(n1, 1)} further step(s) on 1 thread, "
                                          f"{t1s:.1f}s per step"),
                host=dict(cpu=cpu, nproc=os.cpu_count()))


def field_errors(torch, B, wl, prims, dec64, dec32, steps):
    """Per-field max and L1 error of the FP32-mixed path against the FP64 path
    on the GPU, after `steps` steps of the workload from its initial state
    (max |d| / max |FP64|, for the momenta over all three components; L1 =
    sum |d| / sum |FP64|), over all events of the batch."""
    dims = wl["dims"] if isinstance(wl["dims"], list) else [wl["dims"]]
    kind, params = wl["eos"]
    eos = (B.EOS_BAG, params) if kind == "bag" else None
    dt = wl["lam"] * wl["dx"]
    out = {}
    for prec, dec in ((B.FP64, dec64), (B.FP32_MIXED, dec32)):
        s = B.Shasta(dims, wl["dx"], precision=prec, eos=eos)
        if dec is not None:
            s.set_decomposition(dec)
        for k, pr in enumerate(prims):
            s.write_primitive(k, *[torch.from_numpy(a) for a in pr.as_tuple()])
        s.step(dt, steps)
        out[prec] = s
    names = ("E", "Mx", "My", "Mz", "R")
    dmax = [0.0] * 5
    rmax = [0.0] * 5
    dsum = [0.0] * 5
    rsum = [0.0] * 5
    for k in range(len(dims)):
        ref = out[B.FP64].read_conserved(k)
        got = out[B.FP32_MIXED].read_conserved(k)
        for q in range(5):
            d = (got[q] - ref[q]).abs()
            dmax[q] = max(dmax[q], d.max().item())
            rmax[q] = max(rmax[q], ref[q].abs().max().item())
            dsum[q] += d.sum().item()
            rsum[q] += ref[q].abs().sum().item()
    for s in out.values():
        s.close()
    mref = max(rmax[1:4])
    res = {"steps": steps, "against": "GPU FP64 run of the same workload"}
    for q in range(5):
        den = mref if q in (1, 2, 3) else rmax[q]
        res[names[q]] = {"max_rel": dmax[q] / den if den > 0 else dmax[q],
                         "l1_rel": dsum[q] / rsum[q] if rsum[q] > 0 else dsum[q]}
    return res


def leg_record(torch, B, name, steps, warmup, autotune):
    """One precision/batching leg of the metric: throughput, dominant-kernel
    roofline and field error against FP64."""
    s, prims, wl, cells, ms, prof, prec, reps = run_workload(torch, B, name, steps, warmup,
                                                             autotune)
    esize = 8 if prec == B.FP64 else 4
    sw = {k: x for k, x in prof.items() if k.startswith("sweep") and x["launches"]}
    dom = max(sw, key=lambda k: sw[k]["ms_total"])
    per_launch = cells * FIELD_PASSES * esize
    ach = per_launch / (sw[dom]["avg_us"] * 1e-6) / 1e9
    dec = s.decomposition()
    s.close()
    log(f"{name}: measuring the field error against FP64 over {wl['steps']} steps")
    err = field_errors(torch, B, wl, prims, None, dec, wl["steps"])
    return {
        "value": cells * steps / (ms / 1000.0), "unit": "cell-updates/s",
        "ms_per_step": ms / steps, "steps": steps,
        "repeats_ms_per_step": [r / steps for r in reps],
        "dtype": "f32 fields, f64 recovery and sums" if prec == B.FP32_MIXED else "f64",
        "config": {"workload": wl["name"],
                   "grid": wl["dims"] if not isinstance(wl["dims"], list)
                   else f"{len(wl['dims'])} events",
                   "cells": cells, "dx_fm": wl["dx"], "dt_over_dx": wl["lam"],
                   "eos": wl["eos"][0], "precision": wl["precision"]},
        "roofline": {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": ach / HBM_PEAK_GBS, "kernel": dom,
                     "kernel_avg_us": sw[dom]["avg_us"], "bytes_per_launch": per_launch,
                     "note": "FP32 fields: the sweeps are bound by VALU issue (unpacked FP32 "
                             "FCT, FP64 recoveries), not by HBM"},
        "decomposition": format_tiles(dec),
        "kernels": prof,
        "error_vs_fp64": err,
    }


def parse_tiles(text):
    """'p0,p1,pers/p0,p1,pers/p0,p1,pers' (x/y/z) -> list of triples."""
    dec = [tuple(int(v) for v in part.split(",")) for part in text.split("/")]
    if len(dec) != 3 or any(len(t) != 3 for t in dec):
        raise SystemExit("--tiles wants three p0,p1,persistent triples separated by '/'")
    return dec


def format_tiles(dec):
    return "/".join(",".join(str(v) for v in t) for t in dec)


def run_workload(torch, B, name, steps, warmup, autotune=True, profile_steps=12, tiles=None,
                 diff=1.0):
    from paper_1206_0919_amd import inputs
    wl = inputs.workload(name)
    precision = B.FP32_MIXED if wl["precision"] == "fp32" else B.FP64
    s, prims, cells = make_state(torch, B, wl, precision)
    dt = wl["lam"] * wl["dx"]
    if diff != 1.0:
        s.set_antidiffusion(diff)
    if tiles is not None:
        s.set_decomposition(tiles)
    elif autotune:
        s.step(dt, warmup)   # clocks up before the candidates are timed
        t0 = time.time()
        s.autotune(dt, 4)
        log(f"{name}: autotuned in {time.time() - t0:.1f}s: "
            + format_tiles(s.decomposition()))
    warm_through_cycle(torch, s, dt, warmup)
    log(f"{name}: warmup {warmup} steps and a captured 6-step cycle done; "
        f"timing 5 x {steps} steps")
    # five timed repetitions of exactly `steps` steps; the median is the value
    reps = [time_steps(torch, s, dt, steps) for _ in range(5)]
    ms = sorted(reps)[len(reps) // 2]
    prof = kernel_profile(torch, s, dt, profile_steps)
    return s, prims, wl, cells, ms, prof, precision, reps


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=6)
    ap.add_argument("--workload", default="hotspots200")
    ap.add_argument("--no-legs", action="store_true",
                    help="skip the FP32-mixed (shock256_mixed) and batched (batch96) legs")
    ap.add_argument("--bag400", action="store_true",
                    help="also measure the 400^3 bag-model leg")
    ap.add_argument("--variants", action="store_true",
                    help="also measure the workload without antiflux")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--tiles", default=None,
                    help="fixed decomposition 'p0,p1,persistent' for x/y/z separated "
                         "by '/' (as printed in the JSON line's 'decomposition'); "
                         "skips the autotuner")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(events would shard across GPUs; see the design notes)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1206_0919_amd import binding as B
    assert torch.cuda.is_available(), "bench.py needs a GPU"

    s, prims, wl, cells, ms, prof, precision, reps = run_workload(
        torch, B, args.workload, args.steps, args.warmup, not args.no_autotune,
        tiles=parse_tiles(args.tiles) if args.tiles else None)
    value = cells * args.steps / (ms / 1000.0)
    esize = 8 if precision == B.FP64 else 4
    # dominant kernel: the sweep class with the largest total time
    sweeps = {k: v for k, v in prof.items() if k.startswith("sweep") and v["launches"]}
    dom = max(sweeps, key=lambda k: sweeps[k]["ms_total"])
    per_launch = cells * FIELD_PASSES * esize          # algorithmic bytes
    achieved = per_launch / (sweeps[dom]["avg_us"] * 1e-6) / 1e9
    decomposition = format_tiles(s.decomposition())
    traffic = measured_traffic(dom, args.workload, decomposition)
    copy_gbs = copy_ceiling(torch, B)
    floor = (pattern_floor(torch, B, wl["dims"], precision, decomposition)
             if not isinstance(wl["dims"], list) else None)
    step_bytes = 3 * per_launch
    rec = {
        "metric": "SHASTA cell-updates/s per step (FP64 vs FP32 vs batched), % HBM roofline",
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms / args.steps,
        "repeats": {"steps_each": args.steps,
                    "ms_per_step": [r / args.steps for r in reps],
                    "value_is": "median of the five repetitions"},
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if precision == B.FP64 else "f32 fields, f64 recovery",
        "data": "synthetic",
        "config": {"workload": wl["name"],
                   "grid": wl["dims"] if not isinstance(wl["dims"], list) else "96 events",
                   "cells": cells, "dx_fm": wl["dx"], "dt_over_dx": wl["lam"],
                   "eos": wl["eos"][0], "precision": wl["precision"]},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic, "kernel": dom,
                     "kernel_avg_us": sweeps[dom]["avg_us"],
                     "bytes_per_launch": per_launch,
                     "copy_GBs": copy_gbs, "frac_of_copy": achieved / copy_gbs,
                     "pattern_floor": floor,
                     # the dominant kernel's time against the copy with its own
                     # memory pattern and no arithmetic (y and z sweeps only)
                     "frac_of_pattern": (floor[dom]["avg_us"] / sweeps[dom]["avg_us"]
                                         if floor and dom in floor else None)},
        "step_hbm_frac": value * (step_bytes / cells) / (HBM_PEAK_GBS * 1e9),
        "kernels": prof,
        "decomposition": decomposition,
    }
    red = s.reduce(0)
    rec["check"] = {"nonfinite": red["nonfinite"], "clamp": red["clamp"],
                    "floor": red["floor"], "max_eps": red["max_eps"]}
    if not args.no_legs:
        rec["legs"] = {}
        names = ["shock256_mixed", "batch96"] + (["bag400"] if args.bag400 else [])
        for name in names:
            rec["legs"][name] = leg_record(torch, B, name, args.steps, args.warmup,
                                           not args.no_autotune)
    if args.variants:
        # the paper's runs without anti-flux: same workload, transport only;
        # the difference is the cost of the antiflux and its limiter
        rec["variants"] = {}
        ns, _, _, ncells, nms, nprof, _, _ = run_workload(torch, B, args.workload, args.steps,
                                                          args.warmup, not args.no_autotune,
                                                          diff=0.0)
        rec["variants"][args.workload + "_without_antiflux"] = {
            "value": ncells * args.steps / (nms / 1000.0), "unit": "cell-updates/s",
            "ms_per_step": nms / args.steps, "steps": args.steps,
            "antiflux_share_of_step": 1.0 - (nms / args.steps) / rec["ms_per_step"],
            "kernels": nprof}
        ns.close()
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a bounded sample")
        rec["cpu_baseline"] = cpu_baseline(wl, prims)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
