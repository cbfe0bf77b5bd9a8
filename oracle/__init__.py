"""Python access to the CPU oracle (genasm_oracle.c).

TEST INFRASTRUCTURE ONLY: only the tests, the smoke check and the
benchmark's CPU-baseline leg may import this package. The GPU library never
does, and shares no code with it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "genasm_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

IMPROVED = 0
UNCOMPRESSED = 1
_VARIANTS = {"improved": IMPROVED, "uncompressed": UNCOMPRESSED, IMPROVED: IMPROVED,
             UNCOMPRESSED: UNCOMPRESSED}


class Result(ctypes.Structure):
    _fields_ = [
        ("score", ctypes.c_int32),
        ("ref_begin", ctypes.c_uint32),
        ("ref_end", ctypes.c_uint32),
        ("n_windows", ctypes.c_uint32),
        ("n_ops", ctypes.c_uint32),
        ("status", ctypes.c_int32),
        ("d_min", ctypes.c_int32),
        ("search_col", ctypes.c_uint32),
        ("words_stored", ctypes.c_uint64),
        ("words_read", ctypes.c_uint64),
        ("words_peak", ctypes.c_uint64),
        ("cells_window", ctypes.c_uint64),
        ("cells_search", ctypes.c_uint64),
        ("rows_window", ctypes.c_uint64),
        ("word_ops", ctypes.c_uint64),
    ]


RESULT_DTYPE = np.dtype([(name, np.dtype(ct)) for name, ct in
                         [(f[0], {ctypes.c_int32: "<i4", ctypes.c_uint32: "<u4",
                                  ctypes.c_uint64: "<u8"}[f[1]]) for f in Result._fields_]])
assert RESULT_DTYPE.itemsize == ctypes.sizeof(Result)


def compile_source(src: str, out: str) -> str:
    """gcc, plain -O3 and no target-specific flags, so the library also runs
    on other x86-64 hosts."""
    tmp = out + ".tmp"
    subprocess.check_call(["gcc", "-std=c11", "-O3", "-fPIC", "-shared", "-Wall", "-Wextra",
                           "-Wno-unused-parameter", "-I", HERE, "-o", tmp, src, "-lpthread"])
    os.replace(tmp, out)
    return out


def build(force: bool = True) -> str:
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        compile_source(SRC, LIB)
    return LIB


_lib = None


def load(path: str):
    """Load an oracle build and declare its signatures."""
    L = ctypes.CDLL(path)
    u8p = ctypes.POINTER(ctypes.c_uint8)
    u64p = ctypes.POINTER(ctypes.c_uint64)
    L.oracle_align.argtypes = [ctypes.c_int, u8p, ctypes.c_uint32, u8p, ctypes.c_uint32,
                               ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_char_p,
                               ctypes.c_uint32, ctypes.POINTER(Result)]
    L.oracle_align.restype = ctypes.c_int
    L.oracle_sellers.argtypes = [u8p, ctypes.c_uint32, u8p, ctypes.c_uint32]
    L.oracle_sellers.restype = ctypes.c_int64
    L.oracle_filter.argtypes = [u8p, ctypes.c_uint32, u8p, ctypes.c_uint32, ctypes.c_int32,
                                ctypes.POINTER(ctypes.c_uint32)]
    L.oracle_filter.restype = ctypes.c_int32
    L.oracle_check_cigar.argtypes = [u8p, ctypes.c_uint32, u8p, ctypes.c_uint32,
                                     ctypes.c_uint32, ctypes.c_uint32, ctypes.c_char_p,
                                     ctypes.c_uint32, ctypes.c_int32]
    L.oracle_check_cigar.restype = ctypes.c_int
    L.oracle_batch.argtypes = [ctypes.c_int, u8p, u64p, u8p, u64p, ctypes.c_uint64,
                               ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int,
                               ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_int)]
    L.oracle_batch.restype = ctypes.c_double
    L.oracle_dc_rows.argtypes = [u8p, ctypes.c_uint32, u8p, ctypes.c_uint32, ctypes.c_int32, u64p]
    L.oracle_dc_rows.restype = ctypes.c_int
    return L


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build(force=False)
        _lib = load(LIB)
    return _lib


def _codes(x) -> np.ndarray:
    if isinstance(x, (str, bytes)):
        from workloads.gen import _as_codes
        return _as_codes(x)
    return np.ascontiguousarray(x, dtype=np.uint8)


def _ptr(a, ct=ctypes.c_uint8):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def align(P, T, k: int, W: int = 64, O: int = 24, variant="improved") -> dict:
    """Align one pair; returns score, span, window count, op string and
    the table counters."""
    P = _codes(P)
    T = _codes(T)
    cap = len(P) + len(T) + 1
    ops = ctypes.create_string_buffer(cap)
    res = Result()
    lib().oracle_align(_VARIANTS[variant], _ptr(P), len(P), _ptr(T), len(T), k, W, O, ops, cap,
                       ctypes.byref(res))
    out = {f[0]: getattr(res, f[0]) for f in Result._fields_}
    out["ops"] = ops.raw[:res.n_ops].decode() if res.score >= 0 else ""
    return out


def sellers(P, T) -> int:
    P = _codes(P)
    T = _codes(T)
    return int(lib().oracle_sellers(_ptr(P), len(P), _ptr(T), len(T)))


def filter_pair(P, T, k: int):
    """Pre-alignment filter: (distance, leftmost start) of the best substring
    of T for the whole read P, or (-1, 0) when the distance exceeds k."""
    P, T = _codes(P), _codes(T)
    st = ctypes.c_uint32(0)
    d = int(lib().oracle_filter(_ptr(P), len(P), _ptr(T), len(T), int(k), ctypes.byref(st)))
    assert d >= -1, "oracle_filter: out of memory"
    return (d, int(st.value) if d >= 0 else 0)


def check_cigar(P, T, begin: int, end: int, ops: str, score: int) -> int:
    P = _codes(P)
    T = _codes(T)
    b = ops.encode()
    return int(lib().oracle_check_cigar(_ptr(P), len(P), _ptr(T), len(T), begin, end, b, len(b),
                                        score))


def dc_rows(P, T, K: int) -> np.ndarray:
    """Rows 0..K of the DC recurrence of pattern P (|P| <= 64) over all of T."""
    P = _codes(P)
    T = _codes(T)
    out = np.zeros((K + 1, len(T) + 1), dtype=np.uint64)
    rc = lib().oracle_dc_rows(_ptr(P), len(P), _ptr(T), len(T), K, _ptr(out, ctypes.c_uint64))
    if rc:
        raise ValueError("bad arguments")
    return out


def batch(ps, variant="improved", nthreads: int = 0, k=None, W=None, O=None):
    """Align every pair of a workloads.PairSet. Returns (results structured
    array, ops byte buffer, seconds, threads used). Pair i's ops start at
    read_off[i] + ref_off[i] and number results['n_ops'][i]."""
    reads = np.ascontiguousarray(ps.reads, dtype=np.uint8)
    refs = np.ascontiguousarray(ps.refs, dtype=np.uint8)
    read_off = np.ascontiguousarray(ps.read_off, dtype=np.uint64)
    ref_off = np.ascontiguousarray(ps.ref_off, dtype=np.uint64)
    n = ps.n_pairs
    res = np.zeros(n, dtype=RESULT_DTYPE)
    ops = np.zeros(max(1, int(read_off[-1] + ref_off[-1])), dtype=np.uint8)
    used = ctypes.c_int(0)
    secs = lib().oracle_batch(_VARIANTS[variant], _ptr(reads), _ptr(read_off, ctypes.c_uint64),
                              _ptr(refs), _ptr(ref_off, ctypes.c_uint64), n,
                              ps.k if k is None else k, ps.W if W is None else W,
                              ps.O if O is None else O, nthreads, ops.ctypes.data,
                              res.ctypes.data, ctypes.byref(used))
    return res, ops, secs, used.value


def pair_ops(ps, res, ops, i: int) -> str:
    """The op string of pair i from a batch() result."""
    off = int(ps.read_off[i] + ps.ref_off[i])
    return ops[off:off + int(res["n_ops"][i])].tobytes().decode()
