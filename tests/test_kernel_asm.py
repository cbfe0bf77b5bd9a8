"""Checks on the built gfx950 code of the kernels (no GPU needed): every
kernel is one function with no calls and no private (scratch) segment. The
wavefront-level LDS synchronization of the window kernels assumes that every
access to a group's LDS is a DS instruction, which holds only while the
functions that touch it are inlined into their kernels."""
import os
import re
import shutil
import subprocess

import pytest

from paper_2203_15561_amd import build as hip_build

HIPCC = hip_build.hipcc()


@pytest.fixture(scope="module")
def device_asm(tmp_path_factory):
    if not (os.path.exists(HIPCC) or shutil.which(HIPCC)):
        pytest.skip("hipcc not available")
    out = str(tmp_path_factory.mktemp("asm") / "kernels.s")
    cmd = [HIPCC, *hip_build.HIPCC_FLAGS, "-I", hip_build.INCLUDE, "-I", hip_build.CSRC,
           "--cuda-device-only", "-S", os.path.join(hip_build.CSRC, "kernels.hip"), "-o", out]
    subprocess.check_call(cmd, stderr=subprocess.DEVNULL)
    with open(out) as f:
        return f.read()


def kernel_meta(asm):
    """name -> metadata text of each kernel (the YAML block after '.name:')."""
    blocks = re.split(r"\n\s+- \.", asm.split("amdhsa.kernels:")[1])
    out = {}
    for b in blocks:
        m = re.search(r"\.name:\s+(\S+)", b)
        if m:
            out[m.group(1)] = b
    return out


def test_kernels_make_no_calls(device_asm):
    assert "s_swappc_b64" not in device_asm
    assert "s_setpc_b64" not in device_asm


def test_kernels_use_no_scratch(device_asm):
    meta = kernel_meta(device_asm)
    assert any("k_windows" in k for k in meta)
    for name, text in meta.items():
        m = re.search(r"\.private_segment_fixed_size:\s+(\d+)", text)
        assert m and int(m.group(1)) == 0, name
        m = re.search(r"\.vgpr_spill_count:\s+(\d+)", text)
        assert m and int(m.group(1)) == 0, name
