"""Every kernel the library launches by default runs without scratch memory.

Register spills, and private arrays indexed at run time, go to scratch.
Both cost a memory round trip inside the row loop: a wall closure written
as two branches once became indexed stores and slowed the general kernel
by a third.  This reads the kernel descriptors of the built library's
gfx950 code object (the bundle in its .hip_fatbin section) with the LLVM
tools of the ROCm install, and checks .private_segment_fixed_size."""
import os
import re
import shutil
import subprocess

import pytest

from paper_2403_11167_amd import lbm

LLVM = "/opt/rocm/llvm/bin"

# kernels chosen by the default launch shapes (both EOS, both strip widths)
DEFAULT_LAUNCHED = {
    "P periodic (pipelined, no register cap)": r"k_step_p_pipeILi[01]E(dd|ff)Li(64|256)ELi[01]ELi0EE",
    "P periodic, two steps per launch": r"k_step2_pILi[01]E(dd|ff)Li256ELi[01]EE",
    "FE periodic, two steps per launch": r"k_step2_feILi[01]E(ddLi128|ffLi192)EE",
    "FE FP64 periodic (register target 3)": r"k_step_feILi[01]EddLi(64|256)ELi[01]ELi3ELi0EE",
    "FE FP32 periodic (pipelined, register target 5)": r"k_step_fe_pipeILi[01]EffLi(64|256)ELi[01]ELi5EE",
    "P general (walls, drive)": r"k_step_pILi[01]E(dd|ff)Li(64|256)ELi1ELi0ELi1EE",
    "FE general, velocity pass, A term": r"k_step_feILi[01]E(ddLi(64|256)ELi1ELi3|ffLi(64|256)ELi1ELi5)ELi[123]EE",
    "batched step": r"k_batch_step",
    "observation, init, populations": r"k_obs_|k_init|k_get_pop|k_set_pop",
    "surrogate": r"mlpk",
}


def kernel_scratch():
    tools = [os.path.join(LLVM, t) for t in ("llvm-objcopy", "clang-offload-bundler", "llvm-readelf")]
    if not all(os.path.exists(t) for t in tools):
        pytest.skip("LLVM tools of the ROCm install not found")
    lib = lbm.LIB_PATH
    assert os.path.exists(lib), "build the library first"
    import tempfile
    notes = ""
    with tempfile.TemporaryDirectory() as d:
        fat = os.path.join(d, "fatbin.bin")
        subprocess.run([tools[0], "--dump-section", f".hip_fatbin={fat}", lib,
                        os.path.join(d, "copy.so")], check=True)
        blob = open(fat, "rb").read()
        # one offload bundle per translation unit, each starting with the magic
        magic = b"__CLANG_OFFLOAD_BUNDLE__"
        starts = [m.start() for m in re.finditer(re.escape(magic), blob)]
        assert starts, "no offload bundle in .hip_fatbin"
        for i, a in enumerate(starts):
            b = starts[i + 1] if i + 1 < len(starts) else len(blob)
            part, co = os.path.join(d, f"b{i}.bin"), os.path.join(d, f"co{i}.o")
            open(part, "wb").write(blob[a:b])
            subprocess.run([tools[1], "--unbundle", "--type=o", f"--input={part}",
                            "--targets=hipv4-amdgcn-amd-amdhsa--gfx950", f"--output={co}"],
                           check=True)
            notes += subprocess.run([tools[2], "--notes", co], check=True, capture_output=True,
                                    text=True).stdout
    out, name = {}, None
    for line in notes.splitlines():
        m = re.match(r"\s+\.name:\s+(\S+)", line)
        if m:
            name = m.group(1)
        m = re.match(r"\s+\.private_segment_fixed_size:\s+(\d+)", line)
        if m and name:
            out[name] = int(m.group(1))
            name = None
    return out


def test_default_kernels_use_no_scratch():
    sizes = kernel_scratch()
    assert len(sizes) > 100
    for what, pat in DEFAULT_LAUNCHED.items():
        hits = {k: v for k, v in sizes.items() if re.search(pat, k)}
        assert hits, f"no kernel matches {what}"
        bad = {k: v for k, v in hits.items() if v}
        assert not bad, (what, bad)
