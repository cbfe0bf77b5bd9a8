"""The GPU kernels' logic on the CPU: kernels.hip is built unmodified with g++
against the HIP emulation in tests/emu (lanes as threads, lane-group
barriers for DPP moves, ballots and wave barriers; host AddressSanitizer and
UBSan on) and its outputs are compared with the oracle. No GPU is involved;
this catches indexing and control-flow mistakes in the kernels before they
run on hardware."""
import os
import tempfile

import numpy as np
import pytest

import oracle
from tests._helpers import load_hand_examples, rle
from tests.emu import run as emu
from workloads import gen

pytestmark = pytest.mark.slow


@pytest.fixture(scope="module")
def driver():
    with tempfile.TemporaryDirectory() as tmp:
        yield emu.build(os.path.join(tmp, "emu_driver"))


@pytest.fixture(scope="module")
def debug_driver():
    with tempfile.TemporaryDirectory() as tmp:
        yield emu.build(os.path.join(tmp, "emu_driver_debug"), debug=True)


def expected(ps):
    res, ops, _, _ = oracle.batch(ps)
    return [(int(res["score"][i]), rle(oracle.pair_ops(ps, res, ops, i)) if res["score"][i] >= 0 else "",
             int(res["ref_begin"][i]) if res["score"][i] >= 0 else 0,
             int(res["ref_end"][i]) if res["score"][i] >= 0 else 0, int(res["n_windows"][i]))
            for i in range(ps.n_pairs)]


def emulated(driver, ps, form, hard_row=16, hard_lanes=16, tb_prefetch=0, hard_share=50, compact=1):
    res, cig = emu.run(driver, ps, form, 16, 16, 16, hard_row=hard_row, hard_lanes=hard_lanes,
                       tb_prefetch=tb_prefetch, hard_share=hard_share, compact=compact)
    assert (res["flags"] == 0).all()
    return [(int(r["edit_distance"]), c, int(r["ref_begin"]), int(r["ref_end"]), int(r["n_windows"]))
            for r, c in zip(res, cig)]


def check(driver, ps, form, hard_row=16, hard_lanes=16, tb_prefetch=0, hard_share=50, compact=1):
    want, got = expected(ps), emulated(driver, ps, form, hard_row, hard_lanes, tb_prefetch,
                                       hard_share, compact)
    bad = [i for i in range(ps.n_pairs) if want[i] != got[i]]
    assert not bad, (bad[:5], want[bad[0]], got[bad[0]])


@pytest.mark.parametrize("form", [0, 1, emu.UNIMPROVED])
def test_hand_examples(driver, form):
    for ex in load_hand_examples():
        ps = gen.from_lists("hand", [ex["P"]], [ex["T"]], ex["k"], ex["W"], ex["O"])
        check(driver, ps, form)


def test_unimproved_fuzz_and_edges(driver):
    # the ablation form: every row, four edge words per entry, traceback on edges
    rng = np.random.default_rng(77)
    pairs = gen.fuzz(9090, 12, max_len=110)
    for chunk in range(2):
        W = int(rng.choice([8, 33, 64]))
        O = int(rng.choice(sorted({0, W // 2, W - 1})))
        k = int(rng.choice([3, 64]))
        sub = pairs[chunk * 6:(chunk + 1) * 6]
        ps = gen.from_lists("fuzz", [p[0] for p in sub], [p[1] for p in sub], k, W, O)
        check(driver, ps, emu.UNIMPROVED)
    cases = [("", ""), ("", "ACGT"), ("ACGT", ""), ("A" * 64, "C" * 64), ("T" * 65, "")]
    for k in (0, 64):
        ps = gen.from_lists("edge", [c[0] for c in cases], [c[1] for c in cases], k)
        check(driver, ps, emu.UNIMPROVED)


@pytest.mark.parametrize("hard_row,hard_lanes,compact", [(16, 16, 1), (4, 16, 1), (16, 16, 0),
                                                       (0, 64, 0), (65, 16, 1), (4, 64, 0),
                                                       (0, 32, 0), (4, 32, 0)])
def test_fuzz_batched(driver, hard_row, hard_lanes, compact):
    # hard_row 0 with 64 (32) hard lanes sends every pair through the whole- (half-)
    # wavefront path, whose emulation is slow: fewer and shorter pairs there;
    # compact 16-lane groups keep 32-bit table slices (pairs from the hard
    # queue start deep), compact 0 the 64-bit table
    rng = np.random.default_rng(31 + hard_row)
    n, max_len = {64: (6, 110), 32: (12, 160)}.get(hard_lanes, (30, 250))
    pairs = gen.fuzz(4242 + hard_row, 2 * n, max_len=max_len)
    for chunk in range(2):
        W = int(rng.choice([4, 8, 33, 64]))
        O = int(rng.choice(sorted({0, 1, W // 2, W - 1})))
        k = int(rng.choice([1, 5, 64]))
        sub = pairs[chunk * n:(chunk + 1) * n]
        ps = gen.from_lists("fuzz", [p[0] for p in sub], [p[1] for p in sub], k, W, O)
        check(driver, ps, 1, hard_row, hard_lanes, compact=compact)


def test_edge_cases_batched(driver):
    cases = [("", ""), ("", "ACGT"), ("ACGT", ""), ("A" * 64, "C" * 64), ("G" * 130, "G" * 90),
             ("T" * 65, ""), ("ACGT" * 16, "ACGT" * 16)]
    for k in (0, 3, 64):
        ps = gen.from_lists("edge", [c[0] for c in cases], [c[1] for c in cases], k)
        check(driver, ps, 1)
        check(driver, ps, 1, compact=0)


@pytest.mark.parametrize("hard_row,hard_lanes,tb_prefetch,compact",
                         [(16, 16, 0, 1), (65, 16, 0, 1), (16, 16, 1, 1), (16, 16, 0, 0),
                          (16, 64, 0, 0), (16, 16, 1, 0), (16, 32, 0, 0), (16, 32, 1, 0)])
def test_long_read_prefixes_with_decoy(driver, hard_row, hard_lanes, tb_prefetch, compact):
    # 1,000-base prefixes of a true pair and a decoy pair: the decoy's windows
    # need most of the 64 rows (spilled rows with 16 lanes and past row 31 with
    # 32, the whole-wavefront path with 64)
    ps = gen.make("long10k", 2, start=4)  # pair 4 is a decoy, pair 5 is not
    assert ps.decoy.tolist() == [True, False]
    cut = gen.from_lists("long-prefix", [ps.read(i)[:1000] for i in range(2)],
                         [ps.ref(i)[:1100] for i in range(2)], 64)
    check(driver, cut, 1, hard_row, hard_lanes, tb_prefetch, compact=compact)


@pytest.mark.parametrize("budget,ticks", [(1, 0), (3, 0), (0, 5), (0, 40)])
def test_serving_loop(driver, budget, ticks):
    # the serving form's device side: 6 slots reused by 40 requests, three
    # admitted per iteration, each resident pair advancing at most `budget`
    # windows per iteration or until the iteration's deadline (`ticks` reads
    # of the emulated clock) passes; open CIGAR runs carried across
    # iterations, the kernels keeping the hot, cold and finished lists
    pairs = gen.fuzz(5150 + budget + ticks, 24 if budget == 1 else 16, max_len=260)
    cases = [("", ""), ("", "ACGT"), ("ACGT", ""), ("T" * 65, ""), ("A" * 64, "C" * 64),
             ("G" * 130, "G" * 90)]
    reads = [p[0] for p in pairs] + [c[0] for c in cases]
    refs = [p[1] for p in pairs] + [c[1] for c in cases]
    for k, W, O in ((64, 64, 24), (5, 16, 8)):
        ps = gen.from_lists("serve", reads, refs, k, W, O)
        want = expected(ps)
        res, cig = emu.run(driver, ps, emu.SERVE, 16, 16, 16, window_budget=budget, slots=6,
                           admit_per_iteration=3, ticks=ticks)
        assert (res["flags"] == 0).all()
        got = [(int(r["edit_distance"]), c, int(r["ref_begin"]), int(r["ref_end"]),
                int(r["n_windows"])) for r, c in zip(res, cig)]
        bad = [i for i in range(ps.n_pairs) if want[i] != got[i]]
        assert not bad, (k, W, O, bad[:5], want[bad[0]], got[bad[0]])


def test_filter_kernel(driver):
    # multi-word rows (reads over 64 bases), empty reads and references, k caps
    rng = np.random.default_rng(404)
    reads, refs = [], []
    for m, n in [(0, 5), (3, 0), (1, 1), (64, 70), (65, 90), (130, 150), (40, 300)]:
        r = rng.integers(0, 4, m).astype(np.uint8)
        if n >= m and m and rng.random() < 0.7:
            a = int(rng.integers(0, n - m + 1))
            t = rng.integers(0, 4, n).astype(np.uint8)
            t[a:a + m] = r
            for _ in range(int(rng.integers(0, 6))):
                t[int(rng.integers(0, n))] = int(rng.integers(0, 4))
        else:
            t = rng.integers(0, 4, n).astype(np.uint8)
        reads.append(r)
        refs.append(t)
    ps = gen.from_lists("filter", reads, refs, 10)
    for k in (0, 40):
        dist, start = emu.run_filter(driver, ps, k)
        for i in range(ps.n_pairs):
            want = oracle.filter_pair(ps.read(i), ps.ref(i), k)
            assert (int(dist[i]), int(start[i]) if dist[i] >= 0 else 0) == want, (i, k)


@pytest.mark.parametrize("chunk", [1, 7, 0])
def test_chunked_start_search(driver, chunk):
    # the start search split into reference chunks (1 column each, 7, or the
    # whole reference) combines to the same start row and leftmost column
    # 1-column chunks make one search item per reference column: fewer pairs there
    pairs = gen.fuzz(6161 + chunk, 8 if chunk == 1 else 24, max_len=140)
    ps = gen.from_lists("chunks", [p[0] for p in pairs], [p[1] for p in pairs], 64)
    want = expected(ps)
    res, cig = emu.run(driver, ps, 1, 16, 16, 16, search_chunk=chunk)
    got = [(int(r["edit_distance"]), c, int(r["ref_begin"]), int(r["ref_end"]), int(r["n_windows"]))
           for r, c in zip(res, cig)]
    bad = [i for i in range(ps.n_pairs) if want[i] != got[i]]
    assert not bad, (chunk, bad[:5], want[bad[0]], got[bad[0]])


@pytest.mark.parametrize("form,hard_lanes,compact", [(0, 16, 1), (1, 16, 1), (1, 16, 0), (1, 32, 0)])
def test_debug_build_clean(debug_driver, form, hard_lanes, compact):
    # the debug build's invariant checks pass and its queue audit finds every
    # queued pair taken by exactly one window worker: results as the oracle's
    # with no flags (check() asserts flags == 0)
    pairs = gen.fuzz(8080 + hard_lanes, 16, max_len=200)
    cases = [("", ""), ("", "ACGT"), ("ACGT", ""), ("A" * 64, "C" * 64), ("T" * 65, "")]
    for k, W, O in ((64, 64, 24), (5, 16, 8)):
        ps = gen.from_lists("debug", [p[0] for p in pairs] + [c[0] for c in cases],
                            [p[1] for p in pairs] + [c[1] for c in cases], k, W, O)
        check(debug_driver, ps, form, hard_lanes=hard_lanes, compact=compact)
    ps = gen.make("long10k", 2, start=4)  # a decoy and a true pair, 1,000-base prefixes
    cut = gen.from_lists("long-prefix", [ps.read(i)[:1000] for i in range(2)],
                         [ps.ref(i)[:1100] for i in range(2)], 64)
    check(debug_driver, cut, form, hard_lanes=hard_lanes, compact=compact)


def test_debug_build_flags_broken_layout(debug_driver):
    # a launch layout the library never makes (17 LDS rows for 16-lane groups,
    # so a group's second row block would run past its LDS rows) is caught by
    # the debug build before the access: the pairs that need that block end
    # with the internal flag, every other pair still matches the oracle
    ps = gen.make("long10k", 2, start=4)
    cut = gen.from_lists("long-prefix", [ps.read(i)[:1000] for i in range(2)],
                         [ps.ref(i)[:1100] for i in range(2)], 64)
    pairs = gen.fuzz(9191, 8, max_len=120)
    ps = gen.from_lists("mix", [cut.read(i) for i in range(2)] + [p[0] for p in pairs],
                        [cut.ref(i) for i in range(2)] + [p[1] for p in pairs], 64)
    want = expected(ps)
    res, cig = emu.run(debug_driver, ps, 1, 16, 16, 17, hard_row=65, compact=0)
    flagged = (res["flags"] & 2) != 0
    assert flagged[0], "the decoy's windows need rows past the first block"
    assert ((res["flags"] | 2) == 2).all()
    for i in range(ps.n_pairs):
        if not flagged[i]:
            r = res[i]
            got = (int(r["edit_distance"]), cig[i], int(r["ref_begin"]), int(r["ref_end"]),
                   int(r["n_windows"]))
            assert got == want[i], (i, got, want[i])


@pytest.mark.parametrize("lds_rows", [16, 32])
def test_window_distance_around_spilled_passes(driver, lds_rows):
    # windows whose d* falls in the first spilled pass (kept as 32-bit slices),
    # just past it (that pass computed again with whole words), deeper, and at
    # the last row; substitutions, insertions and deletions spread over the
    # first window
    rng = np.random.default_rng(2718 + lds_rows)
    reads, refs = [], []
    for e in (lds_rows - 2, lds_rows, lds_rows + 3, lds_rows + 15, lds_rows + 16, lds_rows + 20, 63):
        e = min(e, 63)
        r = rng.integers(0, 4, 120).astype(np.uint8)
        t = list(r)
        for pos in sorted(rng.choice(60, size=min(e, 60), replace=False), reverse=True):
            kind = rng.integers(0, 3)
            if kind == 0:
                t[pos] = (t[pos] + 1 + rng.integers(0, 3)) % 4
            elif kind == 1:
                del t[pos]
            else:
                t.insert(pos, int(rng.integers(0, 4)))
        reads.append(r)
        refs.append(np.array(t, dtype=np.uint8))
    ps = gen.from_lists("deep", reads, refs, 64)
    want = expected(ps)
    res, cig = emu.run(driver, ps, 1, 16, 16, lds_rows, hard_row=65, compact=0)
    assert (res["flags"] == 0).all()
    got = [(int(r["edit_distance"]), c, int(r["ref_begin"]), int(r["ref_end"]), int(r["n_windows"]))
           for r, c in zip(res, cig)]
    bad = [i for i in range(ps.n_pairs) if want[i] != got[i]]
    assert not bad, (bad[:5], want[bad[0]], got[bad[0]])


@pytest.mark.parametrize("W,O", [(64, 56), (32, 20)])
def test_deep_windows_small_overlap_step(driver, W, O):
    # decoy windows (three or more DC passes) with W - O under 14, where only the
    # last lane of a group stores the boundary row, and above it; 64-bit tables
    # in 16- and 32-lane groups
    ps = gen.make("long10k", 2, start=4)
    cut = gen.from_lists("deep", [ps.read(i)[:600] for i in range(2)],
                         [ps.ref(i)[:700] for i in range(2)], 64, W, O)
    check(driver, cut, 1, 16, 16, compact=0)
    check(driver, cut, 1, 16, 32, compact=0)
