"""The Python binding's structures match the C header field for field: a
small C++ program built against include/genasm.h prints the size of every
struct and the offset of every field, and the ctypes / numpy layouts must
agree (a mismatch would pass garbage through the C ABI)."""
import ctypes
import os
import subprocess

import pytest

from paper_2203_15561_amd import capi

HERE = os.path.dirname(os.path.abspath(__file__))
INCLUDE = os.path.join(HERE, "..", "include")

# C struct name -> ctypes structure of the binding
STRUCTS = {
    "genasm_result": capi.Result,
    "genasm_launch": capi.Launch,
    "genasm_profile": capi.Profile,
    "genasm_server_config": capi.ServerConfig,
    "genasm_peaks": capi.Peaks,
    "genasm_completion": capi.Completion,
    "genasm_server_stats": capi.ServerStats,
}


def test_struct_layouts_match_header(tmp_path):
    lines = ["#include <cstddef>", "#include <cstdio>", '#include "genasm.h"', "int main() {"]
    for cname, st in STRUCTS.items():
        lines.append(f'    std::printf("{cname} %zu\\n", sizeof({cname}));')
        for f in st._fields_:
            lines.append(f'    std::printf("{cname}.{f[0]} %zu\\n", offsetof({cname}, {f[0]}));')
    for f in capi.COMPLETION_INFO_DTYPE.names:
        lines.append(f'    std::printf("genasm_completion_info.{f} %zu\\n", '
                     f'offsetof(genasm_completion_info, {f}));')
    lines.append('    std::printf("genasm_completion_info %zu\\n", sizeof(genasm_completion_info));')
    lines += ["    return 0;", "}"]
    src = tmp_path / "layout.cpp"
    src.write_text("\n".join(lines) + "\n")
    exe = str(tmp_path / "layout")
    try:
        subprocess.run(["g++", "-std=c++17", "-I", INCLUDE, str(src), "-o", exe], check=True,
                       capture_output=True, text=True)
    except FileNotFoundError:
        pytest.skip("g++ not found")
    got = dict(line.split() for line in subprocess.run([exe], capture_output=True, text=True,
                                                        check=True).stdout.splitlines())
    for cname, st in STRUCTS.items():
        assert int(got[cname]) == ctypes.sizeof(st), cname
        for f in st._fields_:
            assert int(got[f"{cname}.{f[0]}"]) == getattr(st, f[0]).offset, f"{cname}.{f[0]}"
    dt = capi.COMPLETION_INFO_DTYPE
    assert int(got["genasm_completion_info"]) == dt.itemsize
    for f in dt.names:
        assert int(got[f"genasm_completion_info.{f}"]) == dt.fields[f][1], f
