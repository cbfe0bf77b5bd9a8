"""ctypes binding of libgenasm.so (declarations in include/genasm.h).

Argument marshalling only: every step of the alignment runs in the library's
HIP kernels. Loading fails loudly when the library has not been built; there
is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# GENASM_LIB_VARIANT=debug loads the debug build (invariant checks and a queue
# audit, reported as GENASM_FLAG_INTERNAL in the results); the default is the
# release build
LIB_PATH = os.path.join(HERE, "libgenasm_debug.so" if os.environ.get("GENASM_LIB_VARIANT") == "debug"
                        else "libgenasm.so")

OK = 0
E_INVAL = -1
E_ALPHABET = -2
E_NOMEM = -3
E_DEVICE = -4
E_NOSPACE = -5
E_BUSY = -6
E_TOOLONG = -7
E_PINNED = -8
E_SCRATCH = -9

# bytes of the static device scratch of the no-allocation device form
NOALLOC_SCRATCH_BYTES = 128 << 20

FORM_PLAIN = 0
FORM_BATCHED = 1
FORM_UNIMPROVED = 2

FLAG_CIGAR_OVERFLOW = 1
FLAG_INTERNAL = 2

OP_CHARS = "=XID"


class Result(ctypes.Structure):
    _fields_ = [
        ("edit_distance", ctypes.c_int32),
        ("ref_begin", ctypes.c_uint32),
        ("ref_end", ctypes.c_uint32),
        ("n_windows", ctypes.c_uint32),
        ("cigar_off", ctypes.c_uint64),
        ("cigar_len", ctypes.c_uint32),
        ("flags", ctypes.c_uint32),
    ]


RESULT_DTYPE = np.dtype([("edit_distance", "<i4"), ("ref_begin", "<u4"), ("ref_end", "<u4"),
                         ("n_windows", "<u4"), ("cigar_off", "<u8"), ("cigar_len", "<u4"),
                         ("flags", "<u4")])
assert RESULT_DTYPE.itemsize == ctypes.sizeof(Result) == 32


class Launch(ctypes.Structure):
    _fields_ = [
        ("form", ctypes.c_int32),
        ("group_lanes", ctypes.c_int32),
        ("search_lanes", ctypes.c_int32),
        ("lds_rows", ctypes.c_int32),
        ("workers_per_cu", ctypes.c_int32),
        ("lpt_order", ctypes.c_int32),
        ("hard_row", ctypes.c_int32),
        ("hard_lanes", ctypes.c_int32),
        ("tb_prefetch", ctypes.c_int32),
        ("hard_share", ctypes.c_int32),
        ("table_bits", ctypes.c_int32),
        ("search_per_cu", ctypes.c_int32),
    ]


class Profile(ctypes.Structure):
    _fields_ = [
        ("total_ms", ctypes.c_float),
        ("order_ms", ctypes.c_float),
        ("search_ms", ctypes.c_float),
        ("windows_ms", ctypes.c_float),
        ("n_pairs", ctypes.c_uint64),
        ("window_word_ops", ctypes.c_uint64),
        ("search_word_ops", ctypes.c_uint64),
        ("window_cells", ctypes.c_uint64),
        ("search_cells", ctypes.c_uint64),
        ("table_words", ctypes.c_uint64),
        ("tb_reads", ctypes.c_uint64),
        ("window_lane_steps", ctypes.c_uint64),
        ("search_lane_steps", ctypes.c_uint64),
        ("windows", ctypes.c_uint64),
        ("dc_cycles", ctypes.c_uint64),
        ("tb_cycles", ctypes.c_uint64),
        ("pair_cycles", ctypes.c_uint64),
        ("window_workgroups", ctypes.c_uint64),
    ]

    def as_dict(self):
        return {f[0]: getattr(self, f[0]) for f in self._fields_}


class ServerConfig(ctypes.Structure):
    _fields_ = [
        ("k", ctypes.c_int32),
        ("W", ctypes.c_int32),
        ("O", ctypes.c_int32),
        ("max_slots", ctypes.c_uint32),
        ("pool_bases", ctypes.c_uint64),
        ("max_pending", ctypes.c_uint32),
        ("window_budget", ctypes.c_uint32),
        ("use_graph", ctypes.c_int32),
        ("iteration_us", ctypes.c_int32),
        ("cigar_runs", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]


class Peaks(ctypes.Structure):
    _fields_ = [
        ("dc_mix_tops", ctypes.c_double),
        ("int32_tops", ctypes.c_double),
        ("lds_tbps", ctypes.c_double),
        ("hbm_tbps", ctypes.c_double),
        ("shift64_tops", ctypes.c_double),
        ("funnel_tops", ctypes.c_double),
        ("dpp_tops", ctypes.c_double),
        ("compute_units", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]


class Completion(ctypes.Structure):
    _fields_ = [
        ("tag", ctypes.c_uint64),
        ("result", Result),
        ("cigar", ctypes.c_void_p),
        ("submit_ns", ctypes.c_uint64),
        ("admit_ns", ctypes.c_uint64),
        ("done_ns", ctypes.c_uint64),
    ]


class ServerStats(ctypes.Structure):
    _fields_ = [
        ("iterations", ctypes.c_uint64),
        ("submitted", ctypes.c_uint64),
        ("admitted", ctypes.c_uint64),
        ("completed", ctypes.c_uint64),
        ("refused", ctypes.c_uint64),
        ("resident", ctypes.c_uint32),
        ("pending", ctypes.c_uint32),
        ("pool_bases_used", ctypes.c_uint64),
        ("device_ms", ctypes.c_double),
        ("cancelled", ctypes.c_uint64),
    ]


COMPLETION_INFO_DTYPE = np.dtype([("tag", "<u8"), ("result", RESULT_DTYPE), ("submit_ns", "<u8"),
                                  ("admit_ns", "<u8"), ("done_ns", "<u8")])
assert COMPLETION_INFO_DTYPE.itemsize == 64
assert ctypes.sizeof(ServerConfig) == 48 and ctypes.sizeof(Completion) == 72
assert ctypes.sizeof(ServerStats) == 72


# Every symbol include/genasm.h declares.
EXPORTS = [
    "genasm_create", "genasm_destroy", "genasm_last_error", "genasm_strerror",
    "genasm_default_launch", "genasm_batch_align", "genasm_batch_align_dev", "genasm_pack",
    "genasm_pack_dev", "genasm_validate", "genasm_version", "genasm_profile_enable",
    "genasm_profile_read", "genasm_server_create", "genasm_submit", "genasm_poll",
    "genasm_completion_release", "genasm_server_stats_read", "genasm_server_destroy",
    "genasm_now_ns", "genasm_filter", "genasm_filter_dev", "genasm_autotune_dev",
    "genasm_tune_cache_save", "genasm_tune_cache_load", "genasm_tune_cache_size",
    "genasm_profile_pairs", "genasm_unpin", "genasm_batch_align_dev_noalloc",
    "genasm_submit_batch", "genasm_poll_batch", "genasm_measure_peaks", "genasm_cancel",
]

_c = ctypes
_u8p = _c.POINTER(_c.c_uint8)
_u64p = _c.POINTER(_c.c_uint64)
_SIGS = {
    "genasm_create": (_c.c_int, [_c.POINTER(_c.c_void_p), _c.c_int]),
    "genasm_destroy": (None, [_c.c_void_p]),
    "genasm_last_error": (_c.c_char_p, [_c.c_void_p]),
    "genasm_strerror": (_c.c_char_p, [_c.c_int]),
    "genasm_default_launch": (_c.c_int, [_c.c_int32, _c.POINTER(Launch)]),
    "genasm_batch_align": (_c.c_int, [_c.c_void_p, _c.c_char_p, _u64p, _c.c_char_p, _u64p,
                                      _c.c_uint64, _c.c_int32, _c.c_int32, _c.c_int32, _c.c_void_p,
                                      _c.c_void_p, _c.c_uint64, _u64p, _c.POINTER(Launch)]),
    "genasm_batch_align_dev": (_c.c_int, [_c.c_void_p, _c.c_void_p, _c.c_void_p, _c.c_void_p,
                                          _c.c_void_p, _c.c_uint64, _c.c_uint64, _c.c_uint64,
                                          _c.c_int32, _c.c_int32, _c.c_int32,
                                          _c.c_void_p, _c.c_void_p, _c.c_uint64,
                                          _c.POINTER(Launch), _c.c_void_p]),
    "genasm_batch_align_dev_noalloc": (_c.c_int, [_c.c_void_p, _c.c_void_p, _c.c_void_p,
                                                  _c.c_void_p, _c.c_void_p, _c.c_uint64,
                                                  _c.c_uint64, _c.c_uint64, _c.c_int32,
                                                  _c.c_int32, _c.c_int32, _c.c_void_p,
                                                  _c.c_void_p, _c.c_uint64, _c.POINTER(Launch),
                                                  _c.c_void_p]),
    "genasm_pack": (_c.c_int, [_c.c_char_p, _c.c_uint64, _c.c_void_p, _u64p]),
    "genasm_pack_dev": (_c.c_int, [_c.c_void_p, _c.c_void_p, _c.c_uint64, _c.c_void_p,
                                   _c.c_void_p, _c.c_void_p]),
    "genasm_validate": (_c.c_int, [_c.c_char_p, _c.c_uint64, _u64p, _c.c_char_p, _c.c_uint64,
                                   _u64p, _c.c_uint64, _c.c_int32, _c.c_int32, _c.c_int32]),
    "genasm_version": (_c.c_char_p, []),
    "genasm_profile_enable": (_c.c_int, [_c.c_void_p, _c.c_int]),
    "genasm_profile_read": (_c.c_int, [_c.c_void_p, _c.c_void_p]),
    "genasm_server_create": (_c.c_int, [_c.c_void_p, _c.POINTER(ServerConfig),
                                        _c.POINTER(_c.c_void_p)]),
    "genasm_submit": (_c.c_int, [_c.c_void_p, _c.c_char_p, _c.c_uint64, _c.c_char_p, _c.c_uint64,
                                 _c.c_int32, _c.c_int32, _c.c_int32, _c.c_uint64]),
    "genasm_submit_batch": (_c.c_int, [_c.c_void_p, _c.c_void_p, _c.c_void_p, _c.c_void_p,
                                       _c.c_void_p, _c.c_uint64, _c.c_int32, _c.c_int32,
                                       _c.c_int32, _c.c_void_p, _u64p]),
    "genasm_measure_peaks": (_c.c_int, [_c.c_void_p, _c.c_void_p]),
    "genasm_cancel": (_c.c_int, [_c.c_void_p, _c.c_uint64]),
    "genasm_poll": (_c.c_int, [_c.c_void_p, _c.c_void_p, _c.c_int, _c.c_int]),
    "genasm_poll_batch": (_c.c_int, [_c.c_void_p, _c.c_void_p, _c.c_int, _c.c_void_p, _c.c_uint64,
                                     _u64p, _c.c_int]),
    "genasm_completion_release": (None, [_c.POINTER(Completion)]),
    "genasm_server_stats_read": (_c.c_int, [_c.c_void_p, _c.POINTER(ServerStats)]),
    "genasm_server_destroy": (None, [_c.c_void_p]),
    "genasm_now_ns": (_c.c_uint64, []),
    "genasm_autotune_dev": (_c.c_int, [_c.c_void_p, _c.c_void_p, _c.c_void_p, _c.c_void_p,
                                       _c.c_void_p, _c.c_uint64, _c.c_uint64, _c.c_uint64,
                                       _c.c_int32, _c.c_int32, _c.c_int32, _c.c_void_p,
                                       _c.c_void_p, _c.c_uint64, _c.c_int32, _c.c_void_p,
                                       _c.POINTER(Launch), _c.POINTER(_c.c_float)]),
    "genasm_profile_pairs": (_c.c_int, [_c.c_void_p, _c.c_void_p, _c.c_uint64, _u64p]),
    "genasm_unpin": (_c.c_int, [_c.c_void_p]),
    "genasm_tune_cache_save": (_c.c_int, [_c.c_void_p, _c.c_char_p]),
    "genasm_tune_cache_load": (_c.c_int, [_c.c_void_p, _c.c_char_p]),
    "genasm_tune_cache_size": (_c.c_int, [_c.c_void_p]),
    "genasm_filter": (_c.c_int, [_c.c_void_p, _c.c_char_p, _u64p, _c.c_char_p, _u64p, _c.c_uint64,
                                 _c.c_int32, _c.c_void_p, _c.c_void_p]),
    "genasm_filter_dev": (_c.c_int, [_c.c_void_p, _c.c_void_p, _c.c_void_p, _c.c_void_p,
                                     _c.c_void_p, _c.c_uint64, _c.c_uint32, _c.c_int32, _c.c_void_p,
                                     _c.c_void_p, _c.c_void_p]),
}

_lib = None


class GenasmError(RuntimeError):
    def __init__(self, code: int, msg: str = ""):
        self.code = code
        super().__init__(f"genasm error {code} ({strerror(code)}){': ' + msg if msg else ''}")


def _share_torch_hip_runtime():
    """PyTorch-ROCm ships its own HIP runtime. Importing torch first makes the
    dynamic linker resolve this library's libamdhip64.so.7 to torch's copy (same
    soname), so the process holds one HIP runtime and torch device memory is
    valid for the kernels. Loaded in the other order, torch would map a second
    runtime, which then finds no device."""
    try:
        import torch  # noqa: F401
    except ImportError:
        pass


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run `python -m paper_2203_15561_amd.build`")
        _share_torch_hip_runtime()
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def strerror(code: int) -> str:
    return lib().genasm_strerror(code).decode()


def version() -> str:
    return lib().genasm_version().decode()


def default_launch(form: int = FORM_BATCHED) -> Launch:
    L = Launch()
    rc = lib().genasm_default_launch(form, ctypes.byref(L))
    if rc:
        raise GenasmError(rc)
    return L


def make_launch(form: int = FORM_BATCHED, **kw) -> Launch:
    L = default_launch(form)
    for key, val in kw.items():
        setattr(L, key, int(val))
    return L


def _ascii(x) -> bytes:
    if isinstance(x, str):
        return x.encode()
    if isinstance(x, (bytes, bytearray)):
        return bytes(x)
    a = np.asarray(x, dtype=np.uint8)
    return np.frombuffer(b"ACGT", dtype=np.uint8)[a].tobytes()


def _concat(seqs):
    parts = [_ascii(s) for s in seqs]
    off = np.zeros(len(parts) + 1, dtype=np.uint64)
    off[1:] = np.cumsum([len(p) for p in parts], dtype=np.uint64)
    return b"".join(parts), off


def pack(seq) -> np.ndarray:
    """2-bit packing of an ACGT sequence by the library's host packer."""
    b = _ascii(seq)
    out = np.zeros((len(b) + 3) // 4, dtype=np.uint8)
    bad = ctypes.c_uint64(0)
    rc = lib().genasm_pack(b, len(b), out.ctypes.data, ctypes.byref(bad))
    if rc:
        raise GenasmError(rc, f"at byte {bad.value}")
    return out


def validate(reads, refs, k: int, W: int = 64, O: int = 24) -> int:
    r, roff = _concat(reads)
    f, foff = _concat(refs)
    return lib().genasm_validate(r, len(r), roff.ctypes.data_as(_u64p), f, len(f),
                                 foff.ctypes.data_as(_u64p), len(roff) - 1, k, W, O)


def decode_cigar(elems) -> str:
    """Text form of device CIGAR elements."""
    e = np.asarray(elems, dtype=np.uint32)
    return "".join(f"{int(x) >> 2}{OP_CHARS[int(x) & 3]}" for x in e)


class Context:
    """One HIP device context (stream + scratch). Not thread-safe."""

    def __init__(self, device: int = 0):
        self._ctx = ctypes.c_void_p()
        rc = lib().genasm_create(ctypes.byref(self._ctx), device)
        if rc:
            raise GenasmError(rc, "genasm_create: " + lib().genasm_last_error(None).decode())
        self.device = device

    def close(self):
        if self._ctx:
            lib().genasm_destroy(self._ctx)
            self._ctx = ctypes.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001 - interpreter shutdown
            pass

    def unpin(self):
        """Declares that no captured graph uses this context's buffers any more."""
        self._check(lib().genasm_unpin(self._ctx), "genasm_unpin")

    def last_error(self) -> str:
        return lib().genasm_last_error(self._ctx).decode()

    def _check(self, rc: int, what: str):
        if rc:
            raise GenasmError(rc, f"{what}: {self.last_error()}")

    def align(self, reads, refs, k: int, W: int = 64, O: int = 24, launch: Launch | None = None):
        """Host-memory form. Returns (results structured array, list of CIGAR strings)."""
        r, roff = _concat(reads)
        f, foff = _concat(refs)
        out, raw = self.align_buffers(r, roff, f, foff, k, W, O, launch)
        cig = [raw[int(o):int(o) + int(L)].decode() for o, L in zip(out["cigar_off"], out["cigar_len"])]
        return out, cig

    def align_buffers(self, r: bytes, roff, f: bytes, foff, k: int, W: int = 64, O: int = 24,
                      launch: Launch | None = None):
        """Host-memory form on concatenated ASCII streams and uint64 offsets.
        Returns (results structured array, CIGAR text buffer as bytes)."""
        roff = np.ascontiguousarray(roff, dtype=np.uint64)
        foff = np.ascontiguousarray(foff, dtype=np.uint64)
        n = len(roff) - 1
        out = np.zeros(n, dtype=RESULT_DTYPE)
        need = ctypes.c_uint64(0)
        # a run of length L takes at most L + 1 <= 2L characters, and a pair has
        # at most m + n ops: 2 (m + n) characters always suffice
        cap = 2 * (len(r) + len(f)) + 16
        buf = np.empty(cap, dtype=np.uint8)
        rc = lib().genasm_batch_align(self._ctx, r, roff.ctypes.data_as(_u64p), f,
                                      foff.ctypes.data_as(_u64p), n, k, W, O, out.ctypes.data,
                                      buf.ctypes.data, cap, ctypes.byref(need),
                                      ctypes.byref(launch) if launch is not None else None)
        self._check(rc, "genasm_batch_align")
        return out, buf[:need.value].tobytes()

    def align_dev(self, reads2b, read_off, refs2b, ref_off, k: int, W: int = 64, O: int = 24,
                  launch: Launch | None = None, out=None, cigar=None, stream=None,
                  total_read_bases=None, total_ref_bases=None, noalloc: bool = False):
        """Device-memory form on torch tensors (uint8 packed streams, int64
        offsets). Returns (out uint8 tensor [n, 32], cigar int32 tensor).
        noalloc=True calls genasm_batch_align_dev_noalloc (the library's static
        device scratch; out and cigar should then be given too, since
        allocating them here would defeat the purpose)."""
        import torch
        n = read_off.numel() - 1
        if total_read_bases is None:
            total_read_bases = int(read_off[-1] - read_off[0])
        if total_ref_bases is None:
            total_ref_bases = int(ref_off[-1] - ref_off[0])
        if out is None:
            out = torch.empty((max(n, 1), 32), dtype=torch.uint8, device=read_off.device)
        cap = total_read_bases + total_ref_bases
        if cigar is None:
            cigar = torch.empty(max(cap, 1), dtype=torch.int32, device=read_off.device)
        if stream is None:
            stream = torch.cuda.current_stream(read_off.device).cuda_stream
        name = "genasm_batch_align_dev_noalloc" if noalloc else "genasm_batch_align_dev"
        rc = getattr(lib(), name)(
            self._ctx, reads2b.data_ptr(), read_off.data_ptr(), refs2b.data_ptr(),
            ref_off.data_ptr(), n, total_read_bases, total_ref_bases, k, W, O,
            out.data_ptr(), cigar.data_ptr(), cigar.numel(),
            ctypes.byref(launch) if launch is not None else None, stream)
        self._check(rc, name)
        return out, cigar

    def filter(self, reads, refs, k: int):
        """Pre-alignment filter, host form. Returns (dist int32 array, start uint32 array)."""
        r, roff = _concat(reads)
        f, foff = _concat(refs)
        n = len(roff) - 1
        dist = np.zeros(n, dtype=np.int32)
        start = np.zeros(n, dtype=np.uint32)
        rc = lib().genasm_filter(self._ctx, r, roff.ctypes.data_as(_u64p), f,
                                 foff.ctypes.data_as(_u64p), n, k, dist.ctypes.data,
                                 start.ctypes.data)
        self._check(rc, "genasm_filter")
        return dist, start

    def filter_dev(self, reads2b, read_off, refs2b, ref_off, k: int, max_read_len: int,
                   dist=None, start=None, stream=None):
        """Pre-alignment filter, device form on torch tensors."""
        import torch
        n = read_off.numel() - 1
        if dist is None:
            dist = torch.empty(max(n, 1), dtype=torch.int32, device=read_off.device)
        if start is None:
            start = torch.empty(max(n, 1), dtype=torch.int32, device=read_off.device)
        if stream is None:
            stream = torch.cuda.current_stream(read_off.device).cuda_stream
        rc = lib().genasm_filter_dev(self._ctx, reads2b.data_ptr(), read_off.data_ptr(),
                                     refs2b.data_ptr(), ref_off.data_ptr(), n, max_read_len, k,
                                     dist.data_ptr(), start.data_ptr(), stream)
        self._check(rc, "genasm_filter_dev")
        return dist, start

    def autotune_dev(self, reads2b, read_off, refs2b, ref_off, k: int, W: int = 64, O: int = 24,
                     out=None, cigar=None, reps: int = 1, stream=None, total_read_bases=None,
                     total_ref_bases=None):
        """Times the batched-form candidates on this batch; returns (Launch, ms, out, cigar)
        and caches the pick for calls without an explicit launch."""
        import torch
        n = read_off.numel() - 1
        if total_read_bases is None:
            total_read_bases = int(read_off[-1] - read_off[0])
        if total_ref_bases is None:
            total_ref_bases = int(ref_off[-1] - ref_off[0])
        if out is None:
            out = torch.empty((max(n, 1), 32), dtype=torch.uint8, device=read_off.device)
        cap = total_read_bases + total_ref_bases
        if cigar is None:
            cigar = torch.empty(max(cap, 1), dtype=torch.int32, device=read_off.device)
        if stream is None:
            stream = torch.cuda.current_stream(read_off.device).cuda_stream
        best = Launch()
        ms = ctypes.c_float(0.0)
        rc = lib().genasm_autotune_dev(
            self._ctx, reads2b.data_ptr(), read_off.data_ptr(), refs2b.data_ptr(),
            ref_off.data_ptr(), n, total_read_bases, total_ref_bases, k, W, O,
            out.data_ptr(), cigar.data_ptr(), cigar.numel(), reps, stream, ctypes.byref(best),
            ctypes.byref(ms))
        self._check(rc, "genasm_autotune_dev")
        return best, float(ms.value), out, cigar

    def tune_cache_save(self, path: str):
        self._check(lib().genasm_tune_cache_save(self._ctx, path.encode()), "genasm_tune_cache_save")

    def tune_cache_load(self, path: str):
        self._check(lib().genasm_tune_cache_load(self._ctx, path.encode()), "genasm_tune_cache_load")

    def tune_cache_size(self) -> int:
        return int(lib().genasm_tune_cache_size(self._ctx))

    def measure_peaks(self) -> dict:
        """Measured device limits (genasm_measure_peaks)."""
        pk = Peaks()
        self._check(lib().genasm_measure_peaks(self._ctx, ctypes.byref(pk)), "genasm_measure_peaks")
        return {f[0]: getattr(pk, f[0]) for f in Peaks._fields_ if f[0] != "reserved"}

    def profile(self, on=True):
        """on: False/0 off, True/1 stage times and work counters, 2 stage times only."""
        self._check(lib().genasm_profile_enable(self._ctx, int(on)), "genasm_profile_enable")

    def profile_read(self) -> dict:
        pr = Profile()
        self._check(lib().genasm_profile_read(self._ctx, ctypes.byref(pr)), "genasm_profile_read")
        return pr.as_dict()

    PROFILE_FIELDS = ("window_word_ops", "search_word_ops", "window_cells", "search_cells",
                      "table_words", "tb_reads", "window_lane_steps", "search_lane_steps",
                      "windows", "dc_cycles", "tb_cycles", "pair_cycles", "start_clock",
                      "end_clock")

    def profile_pairs(self) -> np.ndarray:
        """Per-pair counters of the last profiled call, shape (n_pairs, 14)."""
        words = ctypes.c_uint64(0)
        rc = lib().genasm_profile_pairs(self._ctx, None, 0, ctypes.byref(words))
        if rc not in (0, E_NOSPACE):
            self._check(rc, "genasm_profile_pairs")
        out = np.zeros(int(words.value), dtype=np.uint64)
        self._check(lib().genasm_profile_pairs(self._ctx, out.ctypes.data, out.size,
                                               ctypes.byref(words)), "genasm_profile_pairs")
        return out.reshape(-1, len(self.PROFILE_FIELDS))

    def pack_dev(self, ascii_dev, packed_dev, bad_dev, stream=None):
        import torch
        if stream is None:
            stream = torch.cuda.current_stream(ascii_dev.device).cuda_stream
        rc = lib().genasm_pack_dev(self._ctx, ascii_dev.data_ptr(), ascii_dev.numel(),
                                   packed_dev.data_ptr(), bad_dev.data_ptr(), stream)
        self._check(rc, "genasm_pack_dev")


def now_ns() -> int:
    return int(lib().genasm_now_ns())


class Server:
    """Serving form: continuous batching of single-pair requests on one
    context (see genasm_server_create)."""

    def __init__(self, ctx: Context, k: int, W: int = 64, O: int = 24, max_slots: int = 0,
                 pool_bases: int = 0, max_pending: int = 0, window_budget: int = 0,
                 use_graph: int = 1, iteration_us: int = 0, cigar_runs: int = 0):
        cfg = ServerConfig(k, W, O, max_slots, pool_bases, max_pending, window_budget, use_graph,
                           iteration_us, cigar_runs, 0)
        self._srv = ctypes.c_void_p()
        rc = lib().genasm_server_create(ctx._ctx, ctypes.byref(cfg), ctypes.byref(self._srv))
        if rc:
            raise GenasmError(rc, "genasm_server_create")
        self.ctx = ctx
        self.k, self.W, self.O = k, W, O
        self.cigar_runs = bool(cigar_runs)
        self._buf = (Completion * 4096)()

    def submit(self, read, ref, tag: int) -> int:
        """Queues one request; returns 0 or a GENASM_E_* code (E_BUSY: back-pressure)."""
        r, f = _ascii(read), _ascii(ref)
        return lib().genasm_submit(self._srv, r, len(r), f, len(f), self.k, self.W, self.O, tag)

    def submit_batch(self, reads2b, read_off, refs2b, ref_off, tags) -> tuple:
        """Queues requests from 2-bit packed numpy streams with base offsets
        (n + 1 each) and n tags; returns (rc, accepted)."""
        reads2b = np.ascontiguousarray(reads2b, dtype=np.uint8)
        refs2b = np.ascontiguousarray(refs2b, dtype=np.uint8)
        read_off = np.ascontiguousarray(read_off, dtype=np.uint64)
        ref_off = np.ascontiguousarray(ref_off, dtype=np.uint64)
        tags = np.ascontiguousarray(tags, dtype=np.uint64)
        acc = ctypes.c_uint64(0)
        rc = lib().genasm_submit_batch(self._srv, reads2b.ctypes.data, read_off.ctypes.data,
                                       refs2b.ctypes.data, ref_off.ctypes.data, len(tags), self.k,
                                       self.W, self.O, tags.ctypes.data, ctypes.byref(acc))
        return rc, int(acc.value)

    def cancel(self, tag: int) -> int:
        """Cancels a waiting or resident request; returns 0 or E_INVAL (no such request)."""
        return lib().genasm_cancel(self._srv, tag)

    def poll(self, max_n: int = 4096, timeout_ms: int = 0) -> list:
        """Completions as dicts; "cigar" is the text, or (cigar_runs) a uint32
        array of run-length elements."""
        n = lib().genasm_poll(self._srv, self._buf, min(max_n, len(self._buf)), timeout_ms)
        if n < 0:
            raise GenasmError(n, "genasm_poll")
        out = []
        for c in self._buf[:n]:
            r = c.result
            if self.cigar_runs:
                cig = np.ctypeslib.as_array((ctypes.c_uint32 * r.cigar_len).from_address(c.cigar)).copy() \
                    if c.cigar and r.cigar_len else np.zeros(0, np.uint32)
            else:
                cig = ctypes.string_at(c.cigar).decode() if c.cigar else ""
            out.append({"tag": c.tag, "edit_distance": r.edit_distance, "ref_begin": r.ref_begin,
                        "ref_end": r.ref_end, "n_windows": r.n_windows, "flags": r.flags,
                        "cigar": cig, "submit_ns": c.submit_ns, "admit_ns": c.admit_ns,
                        "done_ns": c.done_ns})
            lib().genasm_completion_release(ctypes.byref(c))
        return out

    def poll_arrays(self, max_n: int = 65536, timeout_ms: int = 0, runs_cap: int = 1 << 24):
        """Bulk poll: (structured array of completion infos, uint32 run
        elements they index), both numpy."""
        if getattr(self, "_info", None) is None or len(self._info) < max_n:
            self._info = np.zeros(max_n, dtype=COMPLETION_INFO_DTYPE)
        if getattr(self, "_runs", None) is None or len(self._runs) < runs_cap:
            self._runs = np.zeros(runs_cap, dtype=np.uint32)
        used = ctypes.c_uint64(0)
        n = lib().genasm_poll_batch(self._srv, self._info.ctypes.data, max_n, self._runs.ctypes.data,
                                    len(self._runs), ctypes.byref(used), timeout_ms)
        if n == E_NOSPACE:
            self._runs = np.zeros(max(int(used.value), 2 * len(self._runs)), dtype=np.uint32)
            return self.poll_arrays(max_n, timeout_ms, len(self._runs))
        if n < 0:
            raise GenasmError(n, "genasm_poll_batch")
        return self._info[:n].copy(), self._runs[:used.value].copy()

    def stats(self) -> dict:
        st = ServerStats()
        rc = lib().genasm_server_stats_read(self._srv, ctypes.byref(st))
        if rc:
            raise GenasmError(rc, "genasm_server_stats_read")
        return {f[0]: getattr(st, f[0]) for f in ServerStats._fields_}

    def close(self):
        if self._srv:
            lib().genasm_server_destroy(self._srv)
            self._srv = ctypes.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001 - interpreter shutdown
            pass
