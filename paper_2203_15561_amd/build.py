"""Builds libgenasm.so (the HIP kernels and the C-ABI runtime) for gfx950.

Run as ``python -m paper_2203_15561_amd.build``; it always recompiles.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libgenasm.so")
# debug variant (GENASM_DEBUG): invariant checks before the guarded LDS and
# spill accesses and a queue audit, reported through the pairs' result flags
LIB_DEBUG = os.path.join(HERE, "libgenasm_debug.so")
SOURCES = ["kernels.hip", "runtime.hip", "server.hip", "peaks.hip"]
ARCH = "gfx950"

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-Wall",
    # no packed FP32 instructions anywhere in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    return "hipcc"


def build(verbose: bool = False, extra_flags=None, debug: bool = False) -> str:
    objs = []
    build_dir = os.path.join(HERE, "_build_debug" if debug else "_build")
    os.makedirs(build_dir, exist_ok=True)
    flags = HIPCC_FLAGS + (["-DGENASM_DEBUG"] if debug else []) + list(extra_flags or [])
    lib = LIB_DEBUG if debug else LIB
    for src in SOURCES:
        obj = os.path.join(build_dir, src.replace(".hip", ".o"))
        cmd = [hipcc(), *flags, "-I", INCLUDE, "-I", CSRC, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        objs.append(obj)
    tmp = lib + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs,
           "-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, lib)
    if not debug:
        write_build_info()
    return lib


BUILD_INFO = os.path.join(HERE, "BUILD_INFO.json")


def write_build_info() -> None:
    """Records the source revision the library was built from (the GPU runs
    see the tree without its git history)."""
    import json
    info = {"git": None, "git_dirty": None, "arch": ARCH}
    try:
        rev = subprocess.run(["git", "-C", ROOT, "rev-parse", "HEAD"], capture_output=True,
                             text=True, timeout=10)
        st = subprocess.run(["git", "-C", ROOT, "status", "--porcelain", "--untracked-files=no"],
                            capture_output=True, text=True, timeout=10)
        if rev.returncode == 0:
            info["git"] = rev.stdout.strip()
            info["git_dirty"] = bool(st.stdout.strip())
    except (OSError, subprocess.SubprocessError):
        pass
    with open(BUILD_INFO, "w") as f:
        json.dump(info, f)


if __name__ == "__main__":
    build(verbose="-q" not in sys.argv, debug="--debug" in sys.argv)
