"""Pins of the CPU oracle against facts that do not come from the oracle.

- hand-worked examples (tests/golden/hand_examples.tsv);
- breadth-first edit search on tiny inputs pins the Sellers routine;
- the meaning of every DC bit (prefix-anchored Levenshtein threshold) pins
  the recurrence term by term;
- on single-window inputs the windowed score equals the Sellers distance;
- every CIGAR replays read into reference with the reported edit count and
  is never cheaper than the Sellers distance;
- the improved and uncompressed forms give identical outputs.
"""
import itertools

import numpy as np
import pytest

from tests._helpers import load_hand_examples, rle, codes_to_str
from workloads import gen


def lev(a: str, b: str) -> int:
    """Levenshtein distance, textbook O(|a||b|) table."""
    prev = list(range(len(b) + 1))
    for i in range(1, len(a) + 1):
        cur = [i] + [0] * len(b)
        for j in range(1, len(b) + 1):
            cur[j] = min(prev[j - 1] + (a[i - 1] != b[j - 1]), prev[j] + 1, cur[j - 1] + 1)
        prev = cur
    return prev[-1]


def neighbours(s: str):
    for k in range(len(s)):
        yield s[:k] + s[k + 1:]
        for c in "ACGT":
            if c != s[k]:
                yield s[:k] + c + s[k + 1:]
    for k in range(len(s) + 1):
        for c in "ACGT":
            yield s[:k] + c + s[k:]


def bfs_infix(P: str, T: str) -> int:
    """Fewest single-base edits turning P into some substring of T, found by
    breadth-first search over strings (no DP table involved)."""
    targets = {T[a:b] for a in range(len(T) + 1) for b in range(a, len(T) + 1)}
    frontier, seen, d = {P}, {P}, 0
    while True:
        if frontier & targets:
            return d
        nxt = set()
        for s in frontier:
            for t in neighbours(s):
                if t not in seen and len(t) <= len(T) + 1:
                    seen.add(t)
                    nxt.add(t)
        frontier, d = nxt, d + 1


def rand_str(rng, n):
    return "".join(rng.choice(list("ACGT"), size=n)) if n else ""


# --------------------------------------------------------------------------
# Sellers brute force
# --------------------------------------------------------------------------

def test_sellers_matches_breadth_first_search(oracle_lib):
    rng = np.random.default_rng(7)
    cases = [("", ""), ("A", ""), ("", "ACG"), ("AC", "CA"), ("ACG", "TTT"), ("GATT", "GTAT")]
    cases += [(rand_str(rng, int(rng.integers(0, 4))), rand_str(rng, int(rng.integers(0, 6))))
              for _ in range(40)]
    for P, T in cases:
        assert oracle_lib.sellers(P, T) == bfs_infix(P, T), (P, T)


def test_sellers_closed_forms(oracle_lib):
    rng = np.random.default_rng(8)
    for _ in range(50):
        T = rand_str(rng, int(rng.integers(1, 80)))
        a = int(rng.integers(0, len(T)))
        b = int(rng.integers(a, len(T) + 1))
        assert oracle_lib.sellers(T[a:b], T) == 0  # an exact occurrence costs nothing
        P = rand_str(rng, int(rng.integers(0, 40)))
        assert oracle_lib.sellers(P, "") == len(P)
        assert oracle_lib.sellers("", T) == 0
        s = oracle_lib.sellers(P, T)
        assert 0 <= s <= len(P)
        assert (s == 0) == (P in T)


# --------------------------------------------------------------------------
# Pre-alignment filter: best substring for the whole read
# --------------------------------------------------------------------------

def test_filter_matches_brute_force(oracle_lib):
    # distance: least Levenshtein distance over every substring T[a:b];
    # start: the least a that reaches it; -1 above k
    rng = np.random.default_rng(17)
    for _ in range(300):
        P = rand_str(rng, int(rng.integers(0, 7)))
        T = rand_str(rng, int(rng.integers(0, 10)))
        best = {a: min(lev(P, T[a:b]) for b in range(a, len(T) + 1)) for a in range(len(T) + 1)}
        d = min(best.values())
        a0 = min(a for a, v in best.items() if v == d)
        for k in (0, 1, 3, 10):
            got = oracle_lib.filter_pair(P, T, k)
            assert got == ((d, a0) if d <= k else (-1, 0)), (P, T, k, got, d, a0)


def test_filter_closed_forms(oracle_lib):
    rng = np.random.default_rng(18)
    for _ in range(60):
        T = rand_str(rng, int(rng.integers(1, 200)))
        a = int(rng.integers(0, len(T)))
        b = int(rng.integers(a + 1, len(T) + 1))
        # an exact occurrence costs nothing and starts at its first occurrence
        assert oracle_lib.filter_pair(T[a:b], T, 0) == (0, T.find(T[a:b]))
        P = rand_str(rng, int(rng.integers(0, 60)))
        assert oracle_lib.filter_pair("", T, 0) == (0, 0)
        assert oracle_lib.filter_pair(P, "", len(P)) == (len(P), 0)
        d, _ = oracle_lib.filter_pair(P, T, 1000)
        assert d == oracle_lib.sellers(P, T)
        assert oracle_lib.filter_pair(P, T, d - 1) == (-1, 0) if d > 0 else True


# --------------------------------------------------------------------------
# DC recurrence: every bit against its meaning
# --------------------------------------------------------------------------

def test_dc_bits_mean_prefix_anchored_distance(oracle_lib):
    """R[d][i] bit p is 0 exactly when the pattern suffix of length p+1 can be
    aligned to some prefix of T[i:] with at most d edits."""
    rng = np.random.default_rng(9)
    for _ in range(60):
        m = int(rng.integers(1, 9))
        n = int(rng.integers(0, 11))
        P, T = rand_str(rng, m), rand_str(rng, n)
        K = int(rng.integers(0, m + 2))
        R = oracle_lib.dc_rows(P, T, K)
        for i in range(n + 1):
            for p in range(m):
                best = min(lev(P[m - 1 - p:], T[i:e]) for e in range(i, n + 1))
                for d in range(K + 1):
                    bit = (int(R[d, i]) >> p) & 1
                    assert bit == (0 if best <= d else 1), (P, T, d, i, p)


def test_dc_invariants(oracle_lib):
    rng = np.random.default_rng(10)
    for _ in range(40):
        m = int(rng.integers(1, 65))
        n = int(rng.integers(0, 200))
        P, T = rand_str(rng, m), rand_str(rng, n)
        K = min(64, m + 1)
        R = oracle_lib.dc_rows(P, T, K).astype(object)
        used = (1 << m) - 1
        for d in range(K + 1):
            low = (1 << min(d, 64)) - 1
            for i in range(n + 1):
                assert int(R[d, i]) & low & used == 0  # d insertions absorb d bases
                if d:
                    # zeros of row d-1 are zeros of row d
                    assert int(R[d, i]) & ~int(R[d - 1, i]) & used == 0
        # row 0 is exact matching: the top bit is 0 exactly where P occurs
        for i in range(n + 1):
            hit = ((int(R[0, i]) >> (m - 1)) & 1) == 0
            assert hit == (T[i:i + m] == P), (P, T, i)


def test_equal_bases_make_the_match_edge_valid(oracle_lib):
    """The property the device traceback's match-run shortcut rests on: at a
    valid cell (bit p of R[d][i] is 0) whose read and text bases agree
    (P[m-1-p] == T[i], i < n), the match edge is valid too (p == 0, or bit p-1
    of R[d][i+1] is 0). Checked on every cell of every row of the oracle's DC
    over random and related pairs, windows of every length up to 64 included."""
    rng = np.random.default_rng(77)
    related = gen.fuzz(4242, 400, max_len=140, related=0.9)
    checked = 0
    for t in range(700):
        if t < 400:
            P, T = codes_to_str(related[t][0][:64]), codes_to_str(related[t][1][:200])
        else:
            P, T = rand_str(rng, int(rng.integers(1, 65))), rand_str(rng, int(rng.integers(0, 130)))
        m, n = len(P), len(T)
        if m == 0 or n == 0:
            continue
        K = min(64, m)
        R = oracle_lib.dc_rows(P, T, K)
        used = np.uint64((1 << m) - 1) if m < 64 else np.uint64(~0 & (2**64 - 1))
        eq = {c: sum(1 << q for q in range(m) if P[m - 1 - q] == c) for c in "ACGT"}
        E = np.array([eq[T[i]] for i in range(n)], dtype=np.uint64)
        valid_eq = ~R[:, :n] & E[None, :] & used
        violated = valid_eq & (R[:, 1:] << np.uint64(1))
        assert not violated.any(), (P, T, np.argwhere(violated)[:3])
        checked += int(np.unpackbits(valid_eq.view(np.uint8)).sum())
    assert checked > 5_000_000, checked


# --------------------------------------------------------------------------
# Whole alignments
# --------------------------------------------------------------------------

@pytest.mark.parametrize("variant", ["improved", "uncompressed"])
def test_hand_examples(oracle_lib, variant):
    for ex in load_hand_examples():
        r = oracle_lib.align(ex["P"], ex["T"], ex["k"], ex["W"], ex["O"], variant)
        got = (r["score"], rle(r["ops"]), r["ref_begin"], r["ref_end"], r["n_windows"])
        want = (ex["score"], ex["cigar"], ex["begin"], ex["end"], ex["windows"])
        assert r["status"] == 0
        assert got == want, (ex, got)


def _check_pair(oracle_lib, P, T, k, W, O, exact_single_window):
    imp = oracle_lib.align(P, T, k, W, O, "improved")
    unc = oracle_lib.align(P, T, k, W, O, "uncompressed")
    assert imp["status"] == 0 and unc["status"] == 0, (imp["status"], unc["status"])
    key = ("score", "ops", "ref_begin", "ref_end", "n_windows")
    assert tuple(imp[x] for x in key) == tuple(unc[x] for x in key), (P, T, k, W, O)
    sel = oracle_lib.sellers(P, T)
    if imp["score"] >= 0:
        assert oracle_lib.check_cigar(P, T, imp["ref_begin"], imp["ref_end"], imp["ops"],
                                      imp["score"]) == 0
        assert imp["score"] >= sel
    if exact_single_window:
        K = min(k, W)
        assert imp["score"] == (sel if sel <= K else -1), (P, T, k, W, O, imp, sel)
    return imp


def test_single_window_equals_sellers(oracle_lib):
    rng = np.random.default_rng(11)
    for W in (64, 33, 8, 4, 2):
        for _ in range(120 if W == 64 else 60):
            m = int(rng.integers(0, W + 1))
            n = int(rng.integers(0, W + 1))
            if rng.random() < 0.5 and m:
                # related pair: a mutated copy with random flanks, clipped to W
                src = rng.integers(0, 4, size=m).astype(np.uint8)
                core = gen.mutate(rng, src, rng.uniform(0, 0.3), (1, 1, 1))
                T = codes_to_str(core)[: W]
                P = codes_to_str(src)
            else:
                P, T = rand_str(rng, m), rand_str(rng, n)
            O = int(rng.integers(0, W))
            k = int(rng.choice([0, 1, 3, 10, 64]))
            _check_pair(oracle_lib, P, T, k, W, O, exact_single_window=True)


def test_improved_equals_uncompressed_fuzz(oracle_lib):
    rng = np.random.default_rng(12)
    pairs = gen.fuzz(1234, 160, max_len=300)
    for idx, (P, T) in enumerate(pairs):
        W = int(rng.choice([4, 8, 16, 32, 63, 64]))
        O = int(rng.choice(sorted({0, 1, W // 2, W - 1})))
        k = int(rng.choice([0, 1, 5, 64]))
        _check_pair(oracle_lib, codes_to_str(P), codes_to_str(T), k, W, O, False)


def test_tiny_windows_many_seams(oracle_lib):
    rng = np.random.default_rng(13)
    for _ in range(80):
        m = int(rng.integers(1, 120))
        src = rng.integers(0, 4, size=m).astype(np.uint8)
        core = gen.mutate(rng, src, rng.uniform(0, 0.25), (1, 1, 1))
        P, T = codes_to_str(src), rand_str(rng, 3) + codes_to_str(core) + rand_str(rng, 3)
        W = int(rng.integers(2, 9))
        O = int(rng.integers(0, W))
        r = _check_pair(oracle_lib, P, T, W, W, O, False)
        assert r["score"] >= 0


def test_k_caps_rows(oracle_lib):
    # the reference has two substitutions inside one window: k=1 fails, k=2 passes
    P = "ACGTACGTAC"
    T = "ACCTACGAAC"
    assert oracle_lib.align(P, T, 1)["score"] == -1
    assert oracle_lib.align(P, T, 2)["score"] == 2
    # k larger than W acts as W
    a = oracle_lib.align(P, T, 64, 8, 2)
    b = oracle_lib.align(P, T, 1000, 8, 2)
    assert (a["score"], a["ops"]) == (b["score"], b["ops"])


def test_row_64_worst_case(oracle_lib):
    # no reference base occurs in the 64-base read: every window needs d* = m_w
    P = "A" * 64
    T = "C" * 64
    r = _check_pair(oracle_lib, P, T, 64, 64, 24, True)
    assert r["score"] == 64
    assert oracle_lib.align(P, T, 63)["score"] == -1


def test_workload_pairs_replay_and_bound(oracle_lib):
    for name, n in (("short100", 30), ("short250", 20), ("uneven", 3)):
        ps = gen.make(name, n)
        res, ops, _, _ = oracle_lib.batch(ps)
        resu, opsu, _, _ = oracle_lib.batch(ps, "uncompressed")
        for i in range(ps.n_pairs):
            P, T = codes_to_str(ps.read(i)), codes_to_str(ps.ref(i))
            o = oracle_lib.pair_ops(ps, res, ops, i)
            assert o == oracle_lib.pair_ops(ps, resu, opsu, i)
            assert res["score"][i] == resu["score"][i]
            assert res["status"][i] == 0
            assert res["score"][i] >= 0
            assert oracle_lib.check_cigar(P, T, int(res["ref_begin"][i]), int(res["ref_end"][i]),
                                          o, int(res["score"][i])) == 0
            assert res["score"][i] >= oracle_lib.sellers(P, T)


@pytest.mark.slow
def test_long_read_lower_bound(oracle_lib):
    ps = gen.make("long10k", 2)
    for i in range(2):
        P, T = ps.read(i), ps.ref(i)
        r = oracle_lib.align(P, T, 64)
        assert r["status"] == 0
        assert oracle_lib.check_cigar(P, T, r["ref_begin"], r["ref_end"], r["ops"], r["score"]) == 0
        assert r["score"] >= oracle_lib.sellers(P, T)


def test_batch_matches_single_calls(oracle_lib):
    ps = gen.make("short100", 40)
    for threads in (1, 3):
        res, ops, secs, used = oracle_lib.batch(ps, nthreads=threads)
        assert used == threads and secs >= 0
        for i in range(ps.n_pairs):
            r = oracle_lib.align(ps.read(i), ps.ref(i), ps.k)
            assert r["score"] == res["score"][i]
            assert r["ops"] == oracle_lib.pair_ops(ps, res, ops, i)


def test_table_footprint_counters(oracle_lib):
    """Improvements 1-3 shrink the stored table: the improved form stores at
    most (d*+1) x (W-O+1) words per window, the uncompressed one 4 words per
    entry for all K+1 rows."""
    ps = gen.make("short250", 10)
    res, _, _, _ = oracle_lib.batch(ps)
    resu, _, _, _ = oracle_lib.batch(ps, "uncompressed")
    assert (res["words_peak"] <= (ps.k + 1) * (ps.W - ps.O + 1)).all()
    assert (resu["words_stored"] > 4 * res["words_stored"]).all()


def test_check_cigar_rejects_wrong_alignments(oracle_lib):
    P, T = "ACGTAC", "TTACGAACTT"
    r = oracle_lib.align(P, T, 64)
    ok = (r["ref_begin"], r["ref_end"], r["ops"], r["score"])
    assert oracle_lib.check_cigar(P, T, *ok) == 0
    b, e, ops, sc = ok
    assert oracle_lib.check_cigar(P, T, b, e, ops, sc + 1) != 0          # wrong edit count
    assert oracle_lib.check_cigar(P, T, b, e, ops[:-1], sc) != 0         # read not consumed
    assert oracle_lib.check_cigar(P, T, b, e + 1, ops, sc) != 0          # span too long
    assert oracle_lib.check_cigar(P, T, b, e, ops.replace("=", "X", 1), sc + 1) != 0  # X on equal
    assert oracle_lib.check_cigar("A", "C", 0, 1, "=", 0) != 0           # = on unequal
    assert oracle_lib.check_cigar("A", "C", 0, 1, "X", 1) == 0
