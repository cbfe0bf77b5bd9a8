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
