"""The chemical potential's logarithms (csrc/lbm_math.h), host build, against
long-double references.

The free-energy step forms mu_b of Eq. 29 (and its van der Waals analogue)
with these functions; parity with the oracle's libm logarithm is checked on
the GPU.  Here the algorithm itself (range reduction, atanh series, ln 2
split, the log1p correction) is pinned to its stated accuracy: within 2 ulp
(FP64 ln) and 3 ulp (FP32 log1p) over the whole range, NaN outside the
domain, exact at 1 and 0.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def errors(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path_factory.mktemp("lbm_math") / "check")
    subprocess.run([gxx, "-O2", "-std=c++17", "-ffp-contract=off",
                    "-I", os.path.join(ROOT, "paper_2403_11167_amd", "csrc"),
                    os.path.join(ROOT, "tests", "lbm_math_check.cpp"), "-o", exe], check=True)
    out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout.split()
    return dict(w64=float(out[0]), w32=float(out[1]), nan_ok=out[2] == "1",
                ln1=float(out[3]), ln1p0=float(out[4]))


def test_ln_f64_within_two_ulp(errors):
    assert errors["w64"] <= 2.0


def test_ln1p_f32_within_three_ulp(errors):
    assert errors["w32"] <= 3.0


def test_domain_and_exact_points(errors):
    assert errors["nan_ok"]
    assert errors["ln1"] == 0.0 and errors["ln1p0"] == 0.0
