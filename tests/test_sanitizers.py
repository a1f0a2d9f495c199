"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU).

The FP64 oracle (every option of its step on small lattices) and the
library's host thermodynamics (thermo.cpp, every entry point) are built
with g++/gcc -fsanitize=address,undefined -fno-sanitize-recover and run;
any out-of-bounds access, leak, use after free, signed overflow or other
undefined behaviour aborts the run.  The GPU code is not built here."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
       "-g", "-O1"]


def _build_and_run(cmd, exe, tmp):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0 and "sanitizer" in (r.stderr or "").lower():
        pytest.skip("sanitizer runtime not available: " + r.stderr[-300:])
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1", OMP_NUM_THREADS="2")
    env.pop("LD_PRELOAD", None)
    out = subprocess.run([exe], capture_output=True, text=True, env=env, cwd=tmp)
    return out


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "orc_san")
    cmd = ["gcc", *SAN, "-fopenmp", "-ffp-contract=off", "-std=c11",
           os.path.join(ROOT, "tests", "sanitize_oracle.c"), "-o", exe, "-lm"]
    out = _build_and_run(cmd, exe, tmp_path)
    assert out.returncode == 0 and out.stdout.strip() == "0", out.stdout + out.stderr[-3000:]


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_host_theory_under_sanitizers(tmp_path):
    exe = str(tmp_path / "thermo_san")
    cmd = ["g++", *SAN, "-std=c++17", "-I", os.path.join(ROOT, "include"),
           os.path.join(ROOT, "paper_2403_11167_amd", "csrc", "thermo.cpp"),
           os.path.join(ROOT, "tests", "sanitize_thermo.cpp"), "-o", exe]
    out = _build_and_run(cmd, exe, tmp_path)
    assert out.returncode == 0 and out.stdout.strip() == "0", out.stdout + out.stderr[-3000:]
