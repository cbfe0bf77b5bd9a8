"""CPU checks of the C ABI: the library loads, exports every symbol the
header declares, and its host-side logic (packing, validation, launch
defaults, error strings) behaves as documented. No kernel runs here."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2203_15561_amd as ga
from paper_2203_15561_amd import capi

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include",
                      "genasm.h")


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[\w\s\*]+?\b(genasm_\w+)\s*\(", text, re.M)))


def test_header_declares_the_bound_symbols():
    assert declared_functions() == sorted(capi.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = ga.lib()
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_pack_layout():
    # base b sits in bits 2*(b%4) of byte b/4, A=0 C=1 G=2 T=3, either case
    rng = np.random.default_rng(1)
    for n in (0, 1, 3, 4, 5, 64, 1001):
        codes = rng.integers(0, 4, n).astype(np.uint8)
        text = bytes(np.frombuffer(b"ACGT", np.uint8)[codes])
        if n:
            text = text[: n // 2].lower() + text[n // 2:]
        want = np.zeros((n + 3) // 4, dtype=np.uint8)
        for b, c in enumerate(codes):
            want[b // 4] |= int(c) << (2 * (b % 4))
        assert (ga.pack(text) == want).all()


def test_pack_rejects_other_bytes():
    with pytest.raises(ga.GenasmError) as e:
        ga.pack("ACGTN")
    assert e.value.code == capi.E_ALPHABET


def test_validate_error_codes():
    assert ga.validate(["ACGT"], ["ACGT"], 5) == capi.OK
    assert ga.validate(["ACGT"], ["AxGT"], 5) == capi.E_ALPHABET
    assert ga.validate(["ACGT"], ["ACGT"], -1) == capi.E_INVAL
    assert ga.validate(["ACGT"], ["ACGT"], 5, W=65) == capi.E_INVAL
    assert ga.validate(["ACGT"], ["ACGT"], 5, W=1, O=0) == capi.E_INVAL
    assert ga.validate(["ACGT"], ["ACGT"], 5, W=8, O=8) == capi.E_INVAL
    assert ga.validate(["ACGT"], ["ACGT"], 5, W=8, O=7) == capi.OK
    assert ga.validate([], [], 5) == capi.OK


def test_validate_offsets():
    lib = ga.lib()
    reads = b"ACGTACGT"
    bad_off = np.array([0, 5, 3], dtype=np.uint64)
    good_off = np.array([0, 3, 8], dtype=np.uint64)
    u64p = ctypes.POINTER(ctypes.c_uint64)
    rc = lib.genasm_validate(reads, 8, bad_off.ctypes.data_as(u64p), reads, 8,
                             good_off.ctypes.data_as(u64p), 2, 5, 64, 24)
    assert rc == capi.E_INVAL
    past_end = np.array([0, 3, 9], dtype=np.uint64)
    rc = lib.genasm_validate(reads, 8, past_end.ctypes.data_as(u64p), reads, 8,
                             good_off.ctypes.data_as(u64p), 2, 5, 64, 24)
    assert rc == capi.E_INVAL


def test_launch_defaults_and_strings():
    L = ga.default_launch(ga.FORM_BATCHED)
    assert L.form == ga.FORM_BATCHED and L.group_lanes in (16, 64) and L.lds_rows % L.group_lanes == 0
    assert ga.default_launch(ga.FORM_PLAIN).form == ga.FORM_PLAIN
    for code in range(-7, 1):
        assert capi.strerror(code)
    assert ga.version().startswith("genasm")


def test_decode_cigar():
    assert ga.decode_cigar([(3 << 2) | 0, (1 << 2) | 1, (2 << 2) | 2, (10 << 2) | 3]) == "3=1X2I10D"


def _gpu_present():
    try:
        import torch
        return torch.cuda.device_count() > 0
    except Exception:  # noqa: BLE001
        return False


@pytest.mark.skipif(_gpu_present(), reason="checks the no-device error path")
def test_create_without_device_is_an_error():
    with pytest.raises(ga.GenasmError) as e:
        ga.Context(0)
    assert e.value.code == capi.E_DEVICE


def test_debug_library_exports_every_declared_symbol():
    # the GENASM_DEBUG build (invariant checks, queue audit) keeps the same ABI
    path = os.path.join(os.path.dirname(capi.LIB_PATH), "libgenasm_debug.so")
    lib = ctypes.CDLL(path)
    for name in declared_functions():
        assert hasattr(lib, name), name
