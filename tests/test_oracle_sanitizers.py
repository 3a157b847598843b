"""The CPU oracle under sanitizers: AddressSanitizer + UndefinedBehaviorSanitizer
(gcc) and ThreadSanitizer over its OpenMP split (clang with the LLVM OpenMP
runtime and its TSan tool, which make the runtime's synchronisation visible to
TSan).  oracle/sanitize_main.c drives every call path on small grids, every
EOS and guarded states; a planted race shows that the TSan build does catch
one."""
import os
import shutil
import subprocess

import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(oracle.__file__))
SRC = os.path.join(HERE, "shasta_oracle.c")
MAIN = os.path.join(HERE, "sanitize_main.c")
LLVM = "/opt/rocm/llvm"
CLANG = os.path.join(LLVM, "bin", "clang")
ARCHER = os.path.join(LLVM, "lib", "libarcher.so")
COMMON = ["-O1", "-g", "-fno-omit-frame-pointer", "-std=c99", "-ffp-contract=off", "-fopenmp"]


def _run(cmd, env=None, timeout=300):
    return subprocess.run(cmd, capture_output=True, text=True, env=env, timeout=timeout)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc missing")
def test_oracle_under_address_and_undefined_sanitizers(tmp_path):
    exe = str(tmp_path / "orc_asan")
    b = _run(["gcc", *COMMON, "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
              SRC, MAIN, "-lm", "-o", exe])
    assert b.returncode == 0, b.stderr
    env = dict(os.environ, OMP_NUM_THREADS="4", ASAN_OPTIONS="detect_leaks=1")
    r = _run([exe], env=env)
    assert r.returncode == 0 and "ok" in r.stdout, r.stdout + r.stderr


def _tsan_build(src, exe):
    b = _run([CLANG, *COMMON, "-fsanitize=thread", src, MAIN, "-lm", "-o", exe,
              f"-Wl,-rpath,{LLVM}/lib"])
    assert b.returncode == 0, b.stderr
    env = dict(os.environ, OMP_NUM_THREADS="4", OMP_TOOL_LIBRARIES=ARCHER,
               TSAN_OPTIONS="ignore_noninstrumented_modules=1")
    return _run([exe], env=env)


@pytest.mark.skipif(not (os.path.exists(CLANG) and os.path.exists(ARCHER)),
                    reason="clang with the LLVM OpenMP TSan tool missing")
def test_oracle_openmp_split_under_thread_sanitizer(tmp_path):
    r = _tsan_build(SRC, str(tmp_path / "orc_tsan"))
    assert r.returncode == 0 and "ok" in r.stdout, r.stdout + r.stderr
    assert "ThreadSanitizer" not in r.stderr


@pytest.mark.skipif(not (os.path.exists(CLANG) and os.path.exists(ARCHER)),
                    reason="clang with the LLVM OpenMP TSan tool missing")
def test_thread_sanitizer_catches_a_planted_race(tmp_path):
    # the per-thread guard counters are merged with atomic additions; without
    # them the merge is a race the TSan build must report
    text = open(SRC).read()
    old = "#pragma omp atomic\n#endif\n    tot.clamp += cnt.clamp;"
    assert old in text
    bad = tmp_path / "shasta_oracle_race.c"
    bad.write_text(text.replace(old, "#endif\n    tot.clamp += cnt.clamp;"))
    r = _tsan_build(str(bad), str(tmp_path / "orc_race"))
    assert "ThreadSanitizer: data race" in r.stderr
