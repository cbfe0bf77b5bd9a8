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
