"""The serving engine's range allocator (host-side C++), built with g++ and
checked by a randomized run against a plain model of the allocated ranges."""
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "..", "paper_2203_15561_amd", "csrc")


def test_range_alloc_randomized(tmp_path):
    exe = str(tmp_path / "range_alloc_test")
    src = os.path.join(HERE, "alloc", "range_alloc_test.cpp")
    try:
        subprocess.run(["g++", "-O1", "-std=c++17", "-fsanitize=address,undefined", "-I", CSRC,
                        src, "-o", exe], check=True, capture_output=True, text=True)
    except FileNotFoundError:
        pytest.skip("g++ not found")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and r.stdout.strip() == "ok", r.stdout + r.stderr
