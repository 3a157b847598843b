"""Host-side logic of bench.py (no GPU): the kernel-source hash that ties a
committed counter summary to the code it was measured on, the matching of a
summary to a decomposition, and the refusal of more than one GPU."""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_code_tokens_drop_comments_and_layout_only():
    src = 'int a = 1; // note\n/* block\n comment */  int  b =\n\t2;'
    assert bench.code_tokens(src) == "int a = 1; int b = 2;"
    # comment markers inside literals are code
    lit = 'asm volatile("s_waitcnt vmcnt(0) // x" ::: "memory"); char c = \'/\';'
    assert bench.code_tokens(lit) == lit
    # an escaped quote does not end a literal
    assert bench.code_tokens('f("a\\"//b"); // c') == 'f("a\\"//b");'


def test_source_hash_ignores_comments_but_not_code():
    files = {f: open(os.path.join(ROOT, "paper_1206_0919_amd", "csrc", f)).read()
             for f in ("shasta_sweeps.hpp", "shasta_kernels.hip", "shasta_math.hpp",
                       "shasta_internal.hpp")}
    base = bench.kernel_source_hash(lambda f: files[f])
    assert base == bench.kernel_source_hash()
    commented = dict(files)
    commented["shasta_math.hpp"] = "// a new comment\n" + files["shasta_math.hpp"] + "\n/* end */\n"
    assert bench.kernel_source_hash(lambda f: commented[f]) == base
    changed = dict(files)
    changed["shasta_math.hpp"] = files["shasta_math.hpp"].replace("1e-300", "1e-299", 1)
    assert changed["shasta_math.hpp"] != files["shasta_math.hpp"]
    assert bench.kernel_source_hash(lambda f: changed[f]) != base


def test_measured_traffic_matches_hash_and_decomposition(tmp_path, monkeypatch):
    prof = tmp_path / "profiles"
    prof.mkdir()
    code = bench.kernel_source_hash()
    entries = [{"decomposition": "8,0,0/100,1,1/67,64,0", "bytes_per_launch": 1.5e9},
               {"decomposition": "8,0,0/50,1,0/200,1,0", "bytes_per_launch": 1.7e9}]
    for k in "xyz":
        (prof / f"traffic_sweep_{k}_w.json").write_text(
            json.dumps({"source_hash": code, "entries": entries}))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: code)
    # x: any decomposition (the windows are fixed by the grid): first entry
    assert bench.measured_traffic("sweep_x", "w", "32,0,1/1,1,1/1,1,1") == 1.5e9
    # y, z: segment length and lanes must match; the launch mode need not
    assert bench.measured_traffic("sweep_y", "w", "2,0,0/100,1,0/1,1,1") == 1.5e9
    assert bench.measured_traffic("sweep_y", "w", "2,0,0/50,1,1/1,1,1") == 1.7e9
    assert bench.measured_traffic("sweep_y", "w", "2,0,0/67,1,1/1,1,1") is None
    assert bench.measured_traffic("sweep_z", "w", "2,0,0/1,1,1/67,64,1") == 1.5e9
    assert bench.measured_traffic("sweep_z", "w", "2,0,0/1,1,1/200,1,1") == 1.7e9
    assert bench.measured_traffic("sweep_z", "w", "2,0,0/1,1,1/67,32,0") is None
    assert bench.measured_traffic("sweep_x", "other", "8,0,0/1,1,1/1,1,1") is None
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0" * 16)
    assert bench.measured_traffic("sweep_x", "w", "8,0,0/1,1,1/1,1,1") is None


def test_bench_refuses_more_than_one_gpu():
    # one GPU is in scope: the benchmark says so and exits before any GPU work
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)
