"""Build ``liblbm.so`` (gfx950 HIP kernels + C ABI + host thermodynamics).

    python -m paper_2403_11167_amd.build

The library is built in-tree next to this file.  Every HIP source is compiled
with packed-FP32 instructions disabled (``-packed-fp32-ops``): plain float
code is all the kernels need and the packed forms are avoided on purpose.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

_HERE = os.path.dirname(os.path.abspath(__file__))
_ROOT = os.path.dirname(_HERE)
SOURCES = [os.path.join(_HERE, "csrc", "lbm_kernels.hip"),
           os.path.join(_HERE, "csrc", "mlp_kernels.hip"),
           os.path.join(_HERE, "csrc", "thermo.cpp")]
OUT = os.path.join(_HERE, "liblbm.so")
DEMO_SRC = os.path.join(_HERE, "csrc", "lbm_cdemo.c")
DEMO = os.path.join(_HERE, "lbm_cdemo")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False) -> str:
    cmd = [hipcc(), "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I", os.path.join(_ROOT, "include"), *SOURCES, "-o", OUT + ".tmp"]
    if verbose:
        print(" ".join(cmd))
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed")
    os.replace(OUT + ".tmp", OUT)
    build_demo(verbose)
    return OUT


def build_demo(verbose: bool = False) -> str:
    """The plain C client of the C ABI (csrc/lbm_cdemo.c), linked against
    liblbm.so next to it and the HIP runtime."""
    cmd = [shutil.which("gcc") or "gcc", "-O2", "-std=c11", "-D__HIP_PLATFORM_AMD__",
           "-I", os.path.join(ROCM, "include"), "-I", os.path.join(_ROOT, "include"), DEMO_SRC,
           "-L", _HERE, "-llbm", "-L", os.path.join(ROCM, "lib"), "-lamdhip64", "-lm",
           "-Wl,-rpath,$ORIGIN", "-Wl,-rpath," + os.path.join(ROCM, "lib"), "-o", DEMO + ".tmp"]
    if verbose:
        print(" ".join(cmd))
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("gcc failed on the C ABI client")
    os.replace(DEMO + ".tmp", DEMO)
    return DEMO


if __name__ == "__main__":
    print(build(verbose=True))
