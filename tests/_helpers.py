"""Helpers shared by the tests (no alignment arithmetic here)."""
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def rle(ops: str) -> str:
    """Run-length form of an op string: '==X' -> '2=1X'."""
    out = []
    k = 0
    while k < len(ops):
        j = k
        while j < len(ops) and ops[j] == ops[k]:
            j += 1
        out.append(f"{j - k}{ops[k]}")
        k = j
    return "".join(out)


def unrle(cigar: str) -> str:
    out = []
    num = ""
    for ch in cigar:
        if ch.isdigit():
            num += ch
        else:
            out.append(ch * int(num))
            num = ""
    return "".join(out)


def load_hand_examples():
    rows = []
    with open(os.path.join(GOLDEN, "hand_examples.tsv")) as f:
        for line in f:
            if not line.strip() or line.startswith("#"):
                continue
            P, T, k, W, O, score, cigar, b, e, nwin = line.rstrip("\n").split("\t")
            rows.append(dict(P="" if P == "-" else P, T="" if T == "-" else T, k=int(k), W=int(W),
                             O=int(O), score=int(score), cigar="" if cigar == "*" else cigar,
                             begin=int(b), end=int(e), windows=int(nwin)))
    return rows


def codes_to_str(a) -> str:
    return np.frombuffer(b"ACGT", dtype=np.uint8)[np.asarray(a, dtype=np.uint8)].tobytes().decode()


# ---------------------------------------------------------------------------
# Whole-batch comparison of device results with the oracle (vectorized, so
# that every pair of a full-size workload is compared, CIGAR included)
# ---------------------------------------------------------------------------

_OP_CODE = np.full(256, 255, dtype=np.uint32)
for _c, _v in zip(b"=XID", range(4)):
    _OP_CODE[_c] = _v
_OP_TEXT = np.frombuffer(b"=XID", dtype=np.uint8)


def oracle_run_elements(ps, res, ops, lo: int, hi: int):
    """Run-length elements (length << 2 | op) of the oracle's op strings of
    pairs lo..hi-1, concatenated in pair order, and the count per pair (0 for
    failed pairs)."""
    n = res["n_ops"][lo:hi].astype(np.int64)
    n[res["score"][lo:hi] < 0] = 0
    base = (ps.read_off[lo:hi] + ps.ref_off[lo:hi]).astype(np.int64)
    segs = [ops[b:b + c] for b, c in zip(base.tolist(), n.tolist()) if c]
    if not segs:
        return np.zeros(0, np.uint32), np.zeros(hi - lo, np.int64)
    codes = _OP_CODE[np.concatenate(segs)]
    assert (codes < 4).all(), "oracle op outside =XID"
    pid = np.repeat(np.arange(hi - lo), n)
    head = np.ones(len(codes), dtype=bool)
    head[1:] = (codes[1:] != codes[:-1]) | (pid[1:] != pid[:-1])
    st = np.flatnonzero(head)
    length = np.diff(np.append(st, len(codes))).astype(np.uint32)
    el = (length << 2) | codes[st]
    return el, np.bincount(pid[st], minlength=hi - lo).astype(np.int64)


def device_run_elements(res, elems, lo: int, hi: int):
    """CIGAR elements of device results lo..hi-1 (cigar_off / cigar_len index
    `elems`), concatenated in pair order, and the count per pair."""
    off = res["cigar_off"][lo:hi].astype(np.int64).tolist()
    cnt = res["cigar_len"][lo:hi].astype(np.int64)
    segs = [elems[o:o + c] for o, c in zip(off, cnt.tolist()) if c]
    el = np.concatenate(segs).astype(np.uint32) if segs else np.zeros(0, np.uint32)
    return el, cnt


def text_run_elements(res, text: bytes, lo: int, hi: int):
    """The host form's CIGAR text of results lo..hi-1 as run elements."""
    off = res["cigar_off"][lo:hi].astype(np.int64).tolist()
    cnt = res["cigar_len"][lo:hi].astype(np.int64)
    segs = [text[o:o + c] for o, c in zip(off, cnt.tolist()) if c]
    buf = np.frombuffer(b"".join(segs), dtype=np.uint8)
    isop = (buf < ord("0")) | (buf > ord("9"))
    op_at = np.flatnonzero(isop)
    dig_at = np.flatnonzero(~isop)
    j = np.searchsorted(op_at, dig_at)
    val = (buf[dig_at].astype(np.uint64) - ord("0")) * (10 ** (op_at[j] - 1 - dig_at)).astype(np.uint64)
    length = np.bincount(j, weights=val.astype(np.float64), minlength=len(op_at)).astype(np.uint32)
    el = (length << 2) | _OP_CODE[buf[op_at]]
    ends = np.cumsum(cnt)
    runs = np.diff(np.concatenate(([0], np.cumsum(isop)[ends - 1] if len(buf) else np.zeros(len(cnt), np.int64))))
    return el, runs.astype(np.int64)


def _elements_text(el) -> str:
    return "".join(f"{int(x) >> 2}{chr(_OP_TEXT[int(x) & 3])}" for x in el)


def assert_batch_matches(ps, ores, oops, gres, run_elements, label="", chunk=2000):
    """Every pair's (edit distance, reference span, window count, CIGAR) of a
    device result array equals the oracle's, bit for bit. `run_elements(lo,
    hi)` returns the device's run elements and counts for pairs lo..hi-1."""
    n = ps.n_pairs
    assert len(gres) >= n and len(ores) == n
    gres = gres[:n]
    assert (ores["status"] == 0).all(), "oracle failed on some pair"
    assert (gres["flags"] == 0).all(), f"{label}: flags set on pairs {np.flatnonzero(gres['flags'])[:10]}"
    ok = ores["score"] >= 0
    want = np.stack([ores["score"].astype(np.int64),
                     np.where(ok, ores["ref_begin"], 0).astype(np.int64),
                     np.where(ok, ores["ref_end"], 0).astype(np.int64),
                     ores["n_windows"].astype(np.int64)], axis=1)
    got = np.stack([gres["edit_distance"].astype(np.int64), gres["ref_begin"].astype(np.int64),
                    gres["ref_end"].astype(np.int64), gres["n_windows"].astype(np.int64)], axis=1)
    bad = np.flatnonzero((want != got).any(axis=1))
    if len(bad):
        i = int(bad[0])
        raise AssertionError(f"{label}: {len(bad)} of {n} pairs differ in (score, begin, end, windows);"
                             f" first pair {i} (m={len(ps.read(i))}, n={len(ps.ref(i))}): oracle "
                             f"{want[i].tolist()} device {got[i].tolist()}")
    for lo in range(0, n, chunk):
        hi = min(n, lo + chunk)
        we, wc = oracle_run_elements(ps, ores, oops, lo, hi)
        ge, gc = run_elements(lo, hi)
        if np.array_equal(wc, gc) and np.array_equal(we, ge):
            continue
        ws = np.concatenate(([0], np.cumsum(wc)))
        gs = np.concatenate(([0], np.cumsum(gc)))
        for j in range(hi - lo):
            a, b = we[ws[j]:ws[j + 1]], ge[gs[j]:gs[j + 1]]
            if not np.array_equal(a, b):
                i = lo + j
                raise AssertionError(f"{label}: CIGAR of pair {i} differs (m={len(ps.read(i))}, "
                                     f"n={len(ps.ref(i))}):\n oracle {_elements_text(a)[:300]}\n"
                                     f" device {_elements_text(b)[:300]}")
        raise AssertionError(f"{label}: CIGAR element streams differ in pairs {lo}..{hi - 1}")
