"""GenASM (windowed bit-parallel DC + TB with the three improvements of
Lindegger et al., 2022) on AMD Instinct MI355X (gfx950).

The alignment runs in libgenasm.so (HIP kernels behind a C ABI, declared in
include/genasm.h); this package only marshals arguments.
"""
from .capi import (  # noqa: F401
    Context, GenasmError, Launch, RESULT_DTYPE, FORM_PLAIN, FORM_BATCHED, FORM_UNIMPROVED, EXPORTS,
    default_launch, make_launch, pack, validate, decode_cigar, version, lib, LIB_PATH,
    Server, now_ns,
)
