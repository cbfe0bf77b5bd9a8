"""GPU tests of the serving form (continuous batching through the C ABI):
every completed request equals the oracle bit for bit, whether it ran alone
or in a mix, with or without the captured iteration graph, under slot and
pool pressure; back-pressure and submit-time errors are reported."""
import time

import numpy as np
import pytest

import oracle
import paper_2203_15561_amd as ga
from tests._helpers import rle
from workloads import gen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    c = ga.Context(0)
    yield c
    c.close()


def expected(ps):
    res, ops, _, _ = oracle.batch(ps)
    assert (res["status"] == 0).all()
    out = []
    for i in range(ps.n_pairs):
        sc = int(res["score"][i])
        cig = rle(oracle.pair_ops(ps, res, ops, i)) if sc >= 0 else ""
        out.append((sc, int(res["ref_begin"][i]) if sc >= 0 else 0,
                    int(res["ref_end"][i]) if sc >= 0 else 0, int(res["n_windows"][i]), cig))
    return out


def as_tuple(c):
    assert c["flags"] == 0, c
    return (c["edit_distance"], c["ref_begin"], c["ref_end"], c["n_windows"], c["cigar"])


def drain(srv, tags, timeout_s=120.0):
    """Polls until every tag in `tags` has completed; returns {tag: completion}."""
    want = set(tags)
    got = {}
    deadline = time.time() + timeout_s
    while want - set(got):
        assert time.time() < deadline, f"{len(want - set(got))} requests did not complete"
        for c in srv.poll(timeout_ms=50):
            assert c["tag"] not in got, c["tag"]
            got[c["tag"]] = c
    return got


def submit_all(srv, ps, tags):
    for t, i in zip(tags, range(ps.n_pairs)):
        rc = srv.submit(ps.read(i), ps.ref(i), t)
        assert rc == 0, (t, rc)


def mixed_set():
    ps = gen.make("serving", 160)
    extra = [("", ""), ("", "ACGT"), ("ACGT", ""), ("T" * 65, ""), ("A" * 64, "C" * 64),
             ("G" * 130, "G" * 90), ("ACGT" * 40, "T" + "ACGT" * 40)]
    reads = [ps.read(i) for i in range(ps.n_pairs)] + [e[0] for e in extra]
    refs = [ps.ref(i) for i in range(ps.n_pairs)] + [e[1] for e in extra]
    return gen.from_lists("serving-mix", reads, refs, ps.k, ps.W, ps.O)


@pytest.fixture(scope="module")
def mix():
    ps = mixed_set()
    return ps, expected(ps)


@pytest.mark.parametrize("use_graph", [1, 0])
def test_mix_matches_oracle(ctx, mix, use_graph):
    ps, want = mix
    with ga.Server(ctx, ps.k, ps.W, ps.O, use_graph=use_graph) as srv:
        tags = list(range(1000, 1000 + ps.n_pairs))
        submit_all(srv, ps, tags)
        got = drain(srv, tags)
        st = srv.stats()
    bad = [i for i, t in enumerate(tags) if as_tuple(got[t]) != want[i]]
    assert not bad, (len(bad), bad[:5], want[bad[0]][:4], as_tuple(got[tags[bad[0]]])[:4])
    assert st["completed"] == ps.n_pairs and st["submitted"] == ps.n_pairs
    for t in tags:
        c = got[t]
        assert c["submit_ns"] <= c["admit_ns"] <= c["done_ns"]


def test_alone_equals_in_mix(ctx, mix):
    ps, want = mix
    # long, short, decoy-free and degenerate requests, each run on an idle server
    picks = [i for i in range(ps.n_pairs) if len(ps.read(i)) > 5000][:3]
    picks += [0, 1, ps.n_pairs - 1, ps.n_pairs - 3]
    with ga.Server(ctx, ps.k, ps.W, ps.O) as srv:
        for i in picks:
            assert srv.submit(ps.read(i), ps.ref(i), 7) == 0
            got = drain(srv, [7])
            assert as_tuple(got[7]) == want[i], i
            assert srv.stats()["resident"] == 0


def test_small_slots_and_pools(ctx, mix):
    # three slots, a base pool that holds about two long requests and a window
    # budget of one: admission waits for space, state persists across many
    # iterations, slots are reused
    ps, want = mix
    longest = max(len(ps.read(i)) + len(ps.ref(i)) for i in range(ps.n_pairs))
    pool = 2 * longest + 4096
    with ga.Server(ctx, ps.k, ps.W, ps.O, max_slots=3, pool_bases=pool, window_budget=1) as srv:
        sel = list(range(0, ps.n_pairs, 5))
        sub = ps.subset(np.array(sel))
        tags = list(range(sub.n_pairs))
        submit_all(srv, sub, tags)
        got = drain(srv, tags, timeout_s=240)
        st = srv.stats()
    for j, i in enumerate(sel):
        assert as_tuple(got[j]) == want[i], i
    assert st["pool_bases_used"] == 0 and st["resident"] == 0


def test_back_pressure(ctx):
    ps = gen.make("serving", 64, start=5000)
    want = expected(ps)
    with ga.Server(ctx, ps.k, ps.W, ps.O, max_pending=4, max_slots=2) as srv:
        accepted, refused = {}, 0
        i = 0
        while i < ps.n_pairs:
            rc = srv.submit(ps.read(i), ps.ref(i), i)
            if rc == 0:
                accepted[i] = True
                i += 1
            else:
                assert rc == ga.capi.E_BUSY
                refused += 1
                for c in srv.poll(timeout_ms=5):
                    accepted[c["tag"]] = c
        pend = [t for t, v in accepted.items() if v is True]
        rest = drain(srv, pend, timeout_s=120)
        accepted.update(rest)
        st = srv.stats()
    assert refused > 0 and st["refused"] == refused
    for i in range(ps.n_pairs):
        assert as_tuple(accepted[i]) == want[i], i


def test_submit_errors(ctx):
    with ga.Server(ctx, 10, 64, 24, pool_bases=1 << 16) as srv:
        assert srv.submit("ACGT", "ACNT", 1) == ga.capi.E_ALPHABET
        assert srv.submit("A" * 40_000, "A" * 40_000, 2) == ga.capi.E_TOOLONG
        # k, W and O are fixed per server
        assert ga.capi.lib().genasm_submit(srv._srv, b"ACGT", 4, b"ACGT", 4, 11, 64, 24, 3) == \
            ga.capi.E_INVAL
        assert srv.submit("ACGT", "ACGT", 4) == 0
        got = drain(srv, [4])
        assert as_tuple(got[4]) == (0, 0, 4, 1, "4=")
        assert srv.stats()["submitted"] == 1


def test_many_requests_match_oracle(ctx):
    # 2,500 requests of the serving mix (70% 150 bp, 30% 1-30 kb), all queued
    # at once: every completion equals the oracle, CIGAR included
    ps = gen.make("serving", 2500, start=20000)
    want = expected(ps)
    with ga.Server(ctx, ps.k, ps.W, ps.O) as srv:
        tags = list(range(ps.n_pairs))
        got = {}
        for t in tags:
            while True:
                rc = srv.submit(ps.read(t), ps.ref(t), t)
                if rc != ga.capi.E_BUSY:
                    break
                for c in srv.poll(timeout_ms=1):
                    got[c["tag"]] = c
            assert rc == 0, (t, rc)
        got.update(drain(srv, [t for t in tags if t not in got], timeout_s=240))
        st = srv.stats()
    bad = [t for t in tags if as_tuple(got[t]) != want[t]]
    assert not bad, (len(bad), bad[:5], want[bad[0]][:4], as_tuple(got[bad[0]])[:4])
    assert st["completed"] == ps.n_pairs and st["resident"] == 0


def _run_elements_from_completions(got, tags):
    """Device-style results and concatenated run elements of completions in tag order."""
    res = np.zeros(len(tags), dtype=ga.RESULT_DTYPE)
    parts, off = [], 0
    for j, t in enumerate(tags):
        c = got[t]
        for f in ("edit_distance", "ref_begin", "ref_end", "n_windows", "flags"):
            res[f][j] = c[f]
        el = c["cigar"]
        res["cigar_off"][j] = off
        res["cigar_len"][j] = len(el)
        parts.append(el)
        off += len(el)
    return res, (np.concatenate(parts).astype(np.uint32) if parts else np.zeros(0, np.uint32))


@pytest.mark.parametrize("iteration_us,unaligned", [(0, False), (30, True)])
def test_batch_submit_runs_match_oracle(ctx, iteration_us, unaligned):
    # 5,000 requests of the serving mix queued through genasm_submit_batch from
    # 2-bit packed streams (with every request starting at a base offset that
    # is not a multiple of 4 when `unaligned`), completions carrying run-length
    # elements; with a 30 us window time the long requests run over many
    # iterations, resuming from their device-resident state each time
    from tests._helpers import assert_batch_matches, device_run_elements
    ps = gen.make("serving", 5000, start=40_000)
    ores, oops, _, _ = oracle.batch(ps)
    reads, refs = ps.reads, ps.refs
    roff, foff = ps.read_off.astype(np.uint64), ps.ref_off.astype(np.uint64)
    if unaligned:
        # one to three junk bases before every request's read and reference
        pad = (np.arange(ps.n_pairs) % 3 + 1).astype(np.uint64)
        def spread(seq, off):
            parts = []
            for i in range(ps.n_pairs):
                parts.append(np.full(int(pad[i]), 2, np.uint8))
                parts.append(seq[off[i]:off[i + 1]])
            return np.concatenate(parts)
        r_cat, f_cat = spread(reads, roff), spread(refs, foff)
        starts_r = np.concatenate(([0], np.cumsum(pad + np.diff(roff))))[:-1] + pad
        starts_f = np.concatenate(([0], np.cumsum(pad + np.diff(foff))))[:-1] + pad
        sub_roff = np.stack([starts_r, starts_r + np.diff(roff)], 1)
        sub_foff = np.stack([starts_f, starts_f + np.diff(foff)], 1)
        assert (sub_roff[:, 0] % 4 != 0).any()
    else:
        r_cat, f_cat = reads, refs
        sub_roff = np.stack([roff[:-1], roff[1:]], 1)
        sub_foff = np.stack([foff[:-1], foff[1:]], 1)
    r2, f2 = ga.pack(r_cat), ga.pack(f_cat)
    tags = np.arange(ps.n_pairs, dtype=np.uint64) + 77
    got = {}
    with ga.Server(ctx, ps.k, ps.W, ps.O, iteration_us=iteration_us, cigar_runs=1) as srv:
        i = 0
        deadline = time.time() + 240
        while i < ps.n_pairs:
            assert time.time() < deadline, "submission did not finish"
            j = min(ps.n_pairs, i + 700)
            # requests i..j-1 as one run of offsets, or one request per call
            # when junk bases separate them
            if unaligned:
                acc = 0
                for q in range(i, j):
                    rc, a = srv.submit_batch(r2, sub_roff[q], f2, sub_foff[q], tags[q:q + 1])
                    if a == 0:
                        break
                    acc += a
            else:
                rc, acc = srv.submit_batch(r2, roff[i:j + 1], f2, foff[i:j + 1], tags[i:j])
            assert rc in (0, ga.capi.E_BUSY), rc
            i += acc
            for c in srv.poll(timeout_ms=1 if acc == 0 else 0):
                got[c["tag"]] = c
        got.update(drain(srv, [int(t) for t in tags if int(t) not in got], timeout_s=240))
        st = srv.stats()
    assert st["completed"] == ps.n_pairs and st["resident"] == 0 and st["pool_bases_used"] == 0
    if iteration_us:
        assert st["iterations"] > 20, st
    res, el = _run_elements_from_completions(got, [int(t) for t in tags])
    assert_batch_matches(ps, ores, oops, res, lambda lo, hi: device_run_elements(res, el, lo, hi),
                         f"serving batch submit (window time {iteration_us} us, unaligned {unaligned})")


def test_batch_submit_errors(ctx):
    ps = gen.make("serving", 4, start=3)
    r2, f2 = ga.pack(ps.reads), ga.pack(ps.refs)
    tags = np.arange(4, dtype=np.uint64)
    with ga.Server(ctx, ps.k, ps.W, ps.O, pool_bases=1 << 16) as srv:
        bad = ps.read_off.astype(np.uint64).copy()
        bad[2], bad[3] = bad[3], bad[2]  # decreasing offsets: nothing queued
        rc, acc = srv.submit_batch(r2, bad, f2, ps.ref_off, tags)
        assert rc == ga.capi.E_INVAL and acc == 0
        # k, W and O are fixed per server
        acc_c = ctypes_u64()
        ro, fo = ps.read_off.astype(np.uint64), ps.ref_off.astype(np.uint64)
        assert ga.capi.lib().genasm_submit_batch(
            srv._srv, r2.ctypes.data, ro.ctypes.data, f2.ctypes.data, fo.ctypes.data, 4, ps.k + 1,
            ps.W, ps.O, tags.ctypes.data, acc_c) == ga.capi.E_INVAL
        assert srv.stats()["submitted"] == 0


def ctypes_u64():
    import ctypes
    return ctypes.byref(ctypes.c_uint64(0))


def test_cancel(ctx):
    # four slots, one window per pair per iteration, 300 requests: most wait
    # on the host when cancelled, the first ones are resident. A request
    # cancelled successfully never completes; every other one completes with
    # the oracle's result, and the slots and pools drain.
    ps = gen.make("serving", 300, start=7000)
    want = expected(ps)
    with ga.Server(ctx, ps.k, ps.W, ps.O, max_slots=4, window_budget=1) as srv:
        tags = list(range(ps.n_pairs))
        for t in tags:
            assert srv.submit(ps.read(t), ps.ref(t), t) == 0
        asked = [0, 1, 2, 3] + list(range(5, 300, 7))
        rcs = {t: srv.cancel(t) for t in asked}
        assert set(rcs.values()) <= {0, ga.capi.E_INVAL}
        assert srv.cancel(10_000) == ga.capi.E_INVAL
        cancelled = {t for t, rc in rcs.items() if rc == 0}
        assert len(cancelled) >= 40
        keep = [t for t in tags if t not in cancelled]
        got = drain(srv, keep, timeout_s=240)
        time.sleep(0.2)
        assert not srv.poll(timeout_ms=50)
        st = srv.stats()
    assert not cancelled & set(got)
    assert st["cancelled"] == len(cancelled) and st["completed"] == len(keep)
    assert st["resident"] == 0 and st["pool_bases_used"] == 0
    for t in keep:
        assert as_tuple(got[t]) == want[t], t
