"""Build libshasta.so (HIP, gfx950) in-tree.

    python -m paper_1206_0919_amd.build

Always recompiles.  Flags: -O3, FP contraction off (every fused multiply-add
is explicit in the sources), packed FP32 instructions disabled.  The
translation units (the sweep kernels of each EOS, the other kernels, the
host library) compile in parallel and are linked into one shared library.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIBDIR = os.path.join(HERE, "lib")
LIB = os.path.join(LIBDIR, "libshasta.so")
SOURCES = [os.path.join(CSRC, f) for f in (
    "sweeps_eos0.hip", "sweeps_eos1.hip", "sweeps_eos2.hip", "sweeps_eos3.hip",
    "shasta_kernels.hip", "shasta_host.cpp")]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]


def hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build(extra=(), out: str = LIB, verbose: bool = False) -> str:
    os.makedirs(os.path.dirname(out), exist_ok=True)
    cc = hipcc()
    with tempfile.TemporaryDirectory() as tmpdir:
        objs = [os.path.join(tmpdir, os.path.basename(src) + ".o") for src in SOURCES]

        def compile_one(job):
            src, obj = job
            cmd = [cc, *HIPCC_FLAGS, *extra, "-c", src, "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            subprocess.run(cmd, check=True)

        workers = max(1, min(len(SOURCES), os.cpu_count() or 1))
        with ThreadPoolExecutor(max_workers=workers) as pool:
            list(pool.map(compile_one, zip(SOURCES, objs)))
        tmp = out + ".tmp"
        cmd = [cc, *HIPCC_FLAGS, *extra, "-shared", *objs, "-o", tmp]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    build(sys.argv[1:], verbose=True)
