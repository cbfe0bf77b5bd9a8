"""Runs the GenASM kernels on the CPU through the HIP emulation (host-side
debugging of kernel logic; no GPU involved)."""
import os
import subprocess
import tempfile

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
RESULT_DTYPE = np.dtype([("edit_distance", "<i4"), ("ref_begin", "<u4"), ("ref_end", "<u4"),
                         ("n_windows", "<u4"), ("cigar_off", "<u8"), ("cigar_len", "<u4"),
                         ("flags", "<u4")])


def build(out_path: str, sanitize: bool = True, debug: bool = False) -> str:
    """debug: the GENASM_DEBUG build (invariant checks and the queue audit)."""
    cmd = ["g++", "-std=c++20", "-O1", "-g", "-fno-omit-frame-pointer", "-I", HERE,
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_2203_15561_amd", "csrc"),
           "-x", "c++", os.path.join(HERE, "emu_driver.cpp"), "-o", out_path, "-lpthread"]
    if sanitize:
        cmd[1:1] = ["-fsanitize=address,undefined"]
    if debug:
        cmd[1:1] = ["-DGENASM_DEBUG"]
    subprocess.check_call(cmd)
    return out_path


def pack2b(codes: np.ndarray) -> np.ndarray:
    codes = np.asarray(codes, dtype=np.uint8)
    n = len(codes)
    pad = np.zeros((n + 3) // 4 * 4, dtype=np.uint8)
    pad[:n] = codes
    q = pad.reshape(-1, 4).astype(np.uint8)
    return (q[:, 0] | (q[:, 1] << 2) | (q[:, 2] << 4) | (q[:, 3] << 6)).astype(np.uint8)


SERVE = 2  # the device side of the serving loop (slot reuse, window budget)
UNIMPROVED = 3  # the unimproved (ablation) form
FILTER = 4      # the pre-alignment filter


def run(driver: str, ps, form: int, group_lanes=16, search_lanes=16, lds_rows=16, hard_row=16,
        timeout=600, window_budget=0, slots=0, admit_per_iteration=0, hard_lanes=16,
        search_chunk=37, tb_prefetch=0, hard_share=50, ticks=0, compact=1):
    """Returns (results, list of (op char, length) runs per pair)."""
    reads2b, refs2b = pack2b(ps.reads), pack2b(ps.refs)
    hdr = np.array([form, group_lanes, search_lanes, lds_rows, ps.k, ps.W, ps.O, ps.n_pairs,
                    len(reads2b), len(refs2b), hard_row, window_budget, slots,
                    admit_per_iteration, hard_lanes, search_chunk, tb_prefetch, hard_share, ticks,
                    compact],
                   dtype=np.int64)
    with tempfile.TemporaryDirectory() as tmp:
        fin, fout = os.path.join(tmp, "in.bin"), os.path.join(tmp, "out.bin")
        with open(fin, "wb") as f:
            for a in (hdr, reads2b, refs2b, ps.read_off.astype(np.uint64), ps.ref_off.astype(np.uint64)):
                f.write(np.ascontiguousarray(a).tobytes())
        subprocess.run([driver, fin, fout], check=True, timeout=timeout)
        raw = open(fout, "rb").read()
    n = ps.n_pairs
    res = np.frombuffer(raw[: 32 * n], dtype=RESULT_DTYPE)
    cig = np.frombuffer(raw[32 * n:], dtype=np.uint32)
    out = []
    for r in res:
        e = cig[int(r["cigar_off"]):int(r["cigar_off"]) + int(r["cigar_len"])]
        out.append("".join(f"{int(x) >> 2}{'=XID'[int(x) & 3]}" for x in e))
    return res, out


def run_filter(driver: str, ps, k: int, timeout=600):
    """Returns (distances, starts) of the filter kernel under emulation."""
    reads2b, refs2b = pack2b(ps.reads), pack2b(ps.refs)
    # same header layout as run() (the batched-form fields are unused here)
    hdr = np.array([FILTER, 64, 64, 64, k, ps.W, ps.O, ps.n_pairs, len(reads2b), len(refs2b),
                    65, 0, 0, 0, 16, 0, 0, 100, 0, 0], dtype=np.int64)
    with tempfile.TemporaryDirectory() as tmp:
        fin, fout = os.path.join(tmp, "in.bin"), os.path.join(tmp, "out.bin")
        with open(fin, "wb") as f:
            for a in (hdr, reads2b, refs2b, ps.read_off.astype(np.uint64), ps.ref_off.astype(np.uint64)):
                f.write(np.ascontiguousarray(a).tobytes())
        subprocess.run([driver, fin, fout], check=True, timeout=timeout)
        raw = open(fout, "rb").read()
    n = ps.n_pairs
    return np.frombuffer(raw[:4 * n], dtype=np.int32), np.frombuffer(raw[4 * n:8 * n], dtype=np.uint32)
