"""The library's build flags and the machine code they give (CPU only).

Every HIP source is compiled with packed-FP32 instruction selection off, so no kernel of
the built library may contain a packed float32 add, multiply or FMA; and with MFMA
accumulators in ordinary VGPRs. The second check disassembles the gfx950 code objects of
the in-tree library (built here from this repository's sources) and is skipped when the
library or the ROCm disassembler is absent."""
import os
import re
import shutil
import subprocess

import pytest

from paper_2304_04781_amd import build as B

OBJDUMP = "/opt/rocm/llvm/bin/llvm-objdump"
PACKED_F32 = re.compile(r"\bv_pk_(add|mul|fma)_f32\b")


def test_flags_disable_packed_fp32_and_use_vgpr_accumulators():
    f = B.common_flags()
    i = f.index("-packed-fp32-ops")
    assert f[i - 3:i] == ["-Xclang", "-target-feature", "-Xclang"]
    j = f.index("-amdgpu-mfma-vgpr-form")
    assert f[j - 1] == "-mllvm"
    assert f"--offload-arch={B.ARCH}" in f and B.ARCH == "gfx950"


@pytest.mark.skipif(not (os.path.exists(B.OUT) and os.path.exists(OBJDUMP)),
                    reason="needs the built library and the ROCm disassembler")
def test_built_kernels_have_no_packed_fp32(tmp_path):
    lib = tmp_path / "lib.so"
    shutil.copy(B.OUT, lib)
    # extracts the offload bundles next to the copy
    subprocess.run([OBJDUMP, "--offloading", str(lib)], cwd=tmp_path, capture_output=True, check=True)
    objs = sorted(p for p in tmp_path.iterdir() if p.name.endswith("gfx950"))
    assert objs, "no gfx950 code objects in the library"
    n_mfma = 0
    for p in objs:
        asm = subprocess.run([OBJDUMP, "-d", f"--mcpu={B.ARCH}", str(p)], capture_output=True, text=True,
                             check=True).stdout
        bad = PACKED_F32.findall(asm)
        assert not bad, f"{p.name}: packed float32 instructions {sorted(set(bad))}"
        n_mfma += asm.count("v_mfma_")
    assert n_mfma > 0  # the disassembly did cover the kernels
