"""GPU parity: the HIP path through the C ABI against the CPU oracle, pair by
pair, on score, reference span, window count and CIGAR. The bar is bit-exact
(integer work)."""
import numpy as np
import pytest

import oracle
import paper_2203_15561_amd as ga
from tests._helpers import load_hand_examples, rle, codes_to_str
from workloads import gen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    c = ga.Context(0)
    yield c
    c.close()


def expected(ps, k=None, W=None, O=None):
    res, ops, _, _ = oracle.batch(ps, k=k, W=W, O=O)
    assert (res["status"] == 0).all()
    out = []
    for i in range(ps.n_pairs):
        sc = int(res["score"][i])
        cig = rle(oracle.pair_ops(ps, res, ops, i)) if sc >= 0 else ""
        out.append((sc, int(res["ref_begin"][i]) if sc >= 0 else 0,
                    int(res["ref_end"][i]) if sc >= 0 else 0, int(res["n_windows"][i]), cig))
    return out


def on_gpu(ctx, ps, launch=None, k=None, W=None, O=None):
    reads = [ps.read(i) for i in range(ps.n_pairs)]
    refs = [ps.ref(i) for i in range(ps.n_pairs)]
    res, cig = ctx.align(reads, refs, ps.k if k is None else k, ps.W if W is None else W,
                         ps.O if O is None else O, launch)
    assert (res["flags"] == 0).all(), np.nonzero(res["flags"])[0][:10]
    return [(int(r["edit_distance"]), int(r["ref_begin"]), int(r["ref_end"]), int(r["n_windows"]),
             c) for r, c in zip(res, cig)]


def assert_same(ps, want, got, label=""):
    assert len(want) == len(got)
    bad = [i for i in range(len(want)) if want[i] != got[i]]
    if bad:
        i = bad[0]
        raise AssertionError(
            f"{label}: {len(bad)} of {len(want)} pairs differ; first pair {i} "
            f"(m={len(ps.read(i))}, n={len(ps.ref(i))}):\n oracle {want[i][:4]} {want[i][4][:200]}\n"
            f" gpu    {got[i][:4]} {got[i][4][:200]}")


FORMS = {
    "plain": ga.make_launch(ga.FORM_PLAIN),
    "batched": None,
    "compact": ga.make_launch(ga.FORM_BATCHED, table_bits=32),
    "unimproved": ga.make_launch(ga.FORM_UNIMPROVED),
}


@pytest.mark.parametrize("form", sorted(FORMS))
def test_hand_examples(ctx, form):
    for ex in load_hand_examples():
        res, cig = ctx.align([ex["P"]], [ex["T"]], ex["k"], ex["W"], ex["O"], FORMS[form])
        got = (int(res["edit_distance"][0]), cig[0], int(res["ref_begin"][0]),
               int(res["ref_end"][0]), int(res["n_windows"][0]))
        assert got == (ex["score"], ex["cigar"], ex["begin"], ex["end"], ex["windows"]), ex


@pytest.mark.parametrize("form", sorted(FORMS))
def test_short100_all_pairs(ctx, form):
    ps = gen.make("short100")
    assert_same(ps, expected(ps), on_gpu(ctx, ps, FORMS[form]), f"short100/{form}")


@pytest.mark.parametrize("form", sorted(FORMS))
def test_short250_subset(ctx, form):
    ps = gen.make("short250", 3000)
    assert_same(ps, expected(ps), on_gpu(ctx, ps, FORMS[form]), f"short250/{form}")


@pytest.mark.parametrize("form", sorted(FORMS))
def test_long10k_subset(ctx, form):
    ps = gen.make("long10k", 48)
    assert ps.decoy.any() and not ps.decoy.all()
    assert_same(ps, expected(ps), on_gpu(ctx, ps, FORMS[form]), f"long10k/{form}")


def test_long10k_full_batch(ctx):
    # The headline workload at its full size (20,000 pairs) in the device form with
    # the default launch, as the benchmark runs it: every pair's CIGAR consumes
    # exactly its read and its reported reference span and its edits add up to
    # the reported edit distance; 96 sampled pairs (decoys and true pairs, the
    # first and the last of the batch) equal the oracle exactly.
    import torch
    ps = gen.make("long10k")
    dev = torch.device("cuda:0")
    r2 = torch.from_numpy(ga.pack(ps.reads)).to(dev)
    f2 = torch.from_numpy(ga.pack(ps.refs)).to(dev)
    ro = torch.from_numpy(ps.read_off.astype(np.int64)).to(dev)
    fo = torch.from_numpy(ps.ref_off.astype(np.int64)).to(dev)
    out, cig = ctx.align_dev(r2, ro, f2, fo, ps.k)
    torch.cuda.synchronize()
    res = out.cpu().numpy().view(ga.RESULT_DTYPE).reshape(-1)[:ps.n_pairs]
    el = cig.cpu().numpy().view(np.uint32)
    assert (res["flags"] == 0).all()
    assert (res["edit_distance"] >= 0).all()
    m = np.diff(ps.read_off.astype(np.int64))
    n = np.diff(ps.ref_off.astype(np.int64))
    off = res["cigar_off"].astype(np.int64)
    cnt = res["cigar_len"].astype(np.int64)
    pair = np.repeat(np.arange(ps.n_pairs), cnt)
    start = np.repeat(off - np.concatenate(([0], np.cumsum(cnt)[:-1])), cnt)
    e = el[np.arange(cnt.sum()) + start]
    length, op = (e >> 2).astype(np.int64), e & 3
    read_used = np.bincount(pair, length * (op != 3), ps.n_pairs)
    ref_used = np.bincount(pair, length * (op != 2), ps.n_pairs)
    edits = np.bincount(pair, length * (op != 0), ps.n_pairs)
    span = res["ref_end"].astype(np.int64) - res["ref_begin"].astype(np.int64)
    assert (read_used == m).all()
    assert (ref_used == span).all() and (res["ref_end"] <= n).all()
    assert (edits == res["edit_distance"]).all()
    rng = np.random.default_rng(2024)
    sample = sorted(set([0, 1, ps.n_pairs - 1]) | set(rng.choice(ps.n_pairs, 93, replace=False).tolist()))
    sub = ps.subset(np.array(sample))
    assert sub.decoy.any() and not sub.decoy.all()
    got = [(int(res["edit_distance"][i]), int(res["ref_begin"][i]), int(res["ref_end"][i]),
            int(res["n_windows"][i]), ga.decode_cigar(el[off[i]:off[i] + cnt[i]])) for i in sample]
    assert_same(sub, expected(sub), got, "long10k full batch")


@pytest.mark.parametrize("form", sorted(FORMS))
def test_uneven_subset(ctx, form):
    ps = gen.make("uneven", 300)
    assert_same(ps, expected(ps), on_gpu(ctx, ps, FORMS[form]), f"uneven/{form}")


LAUNCH_VARIANTS = {
    "g64": dict(group_lanes=64, lds_rows=64),
    "g16_rows32": dict(group_lanes=16, lds_rows=32),
    "g16_rows64": dict(group_lanes=16, lds_rows=64),
    "search64": dict(search_lanes=64),
    "input_order": dict(lpt_order=0),
    "one_worker": dict(workers_per_cu=1),
    "all_hard": dict(hard_row=-1),
    "all_hard_g64": dict(hard_row=-1, hard_lanes=64),
    "no_hard": dict(hard_row=65),
    "hard_from_8": dict(hard_row=8),
    "hard_g64": dict(hard_row=16, hard_lanes=64),
    "hard_g32": dict(hard_row=16, hard_lanes=32),
    "all_hard_g32": dict(hard_row=-1, hard_lanes=32),
    "hard_g32_rows48": dict(hard_row=12, hard_lanes=32, lds_rows=48),
    "hard_g32_prefetch": dict(hard_row=16, hard_lanes=32, tb_prefetch=1),
    "tb_prefetch": dict(tb_prefetch=1),
    "hard_share_0": dict(hard_share=0),
    "hard_share_100": dict(hard_share=100),
    "hard_share_30_g32": dict(hard_share=30, hard_lanes=32),
    "hard_share_70_g64": dict(hard_share=70, hard_lanes=64),
    # compact 16-lane groups: 32-bit table slices, deep windows recomputed in device memory
    "compact": dict(table_bits=32),
    "compact_no_hard": dict(table_bits=32, hard_row=65),
    "compact_all_hard": dict(table_bits=32, hard_row=-1),
    "compact_prefetch": dict(table_bits=32, tb_prefetch=1),
    "compact_one_worker": dict(table_bits=32, workers_per_cu=1),
    "search_4_per_cu": dict(search_per_cu=4),
    "search_16_per_cu": dict(search_per_cu=16),
}


@pytest.mark.parametrize("variant", sorted(LAUNCH_VARIANTS))
def test_batched_launch_variants(ctx, variant):
    L = ga.make_launch(ga.FORM_BATCHED, **LAUNCH_VARIANTS[variant])
    ps = gen.make("long10k", 24, start=100)
    assert_same(ps, expected(ps), on_gpu(ctx, ps, L), f"long10k/{variant}")
    ps = gen.make("uneven", 200, start=500)
    assert_same(ps, expected(ps), on_gpu(ctx, ps, L), f"uneven/{variant}")


@pytest.mark.parametrize("form", sorted(FORMS))
def test_fuzz_windows_and_caps(ctx, form):
    rng = np.random.default_rng(21)
    pairs = gen.fuzz(777, 600, max_len=400)
    for chunk in range(6):
        W = int(rng.choice([2, 4, 8, 16, 33, 63, 64]))
        O = int(rng.choice(sorted({0, 1, W // 2, W - 1})))
        k = int(rng.choice([0, 1, 5, 15, 64, 100]))
        sub = pairs[chunk * 100:(chunk + 1) * 100]
        ps = gen.from_lists("fuzz", [p[0] for p in sub], [p[1] for p in sub], k, W, O)
        assert_same(ps, expected(ps), on_gpu(ctx, ps, FORMS[form]), f"fuzz W={W} O={O} k={k}/{form}")


@pytest.mark.parametrize("form", sorted(FORMS))
def test_edge_cases(ctx, form):
    cases = [
        ("", ""), ("", "ACGT"), ("ACGT", ""), ("A", "A"), ("A", "C"), ("A" * 64, "C" * 64),
        ("A" * 64, "C" * 200), ("ACGT" * 16, "ACGT" * 16), ("ACGT" * 40, "T" + "ACGT" * 40),
        ("G" * 130, "G" * 90), ("T" * 65, ""), ("ACGTTGCA" * 100, "ACGTTGCA" * 100),
    ]
    for k in (0, 3, 64):
        ps = gen.from_lists("edge", [c[0] for c in cases], [c[1] for c in cases], k)
        assert_same(ps, expected(ps), on_gpu(ctx, ps, FORMS[form]), f"edge k={k}/{form}")


def test_device_form_matches_host_form(ctx):
    import torch
    ps = gen.make("uneven", 64)
    res_h, cig_h = ctx.align([ps.read(i) for i in range(ps.n_pairs)],
                             [ps.ref(i) for i in range(ps.n_pairs)], ps.k)
    dev = torch.device("cuda:0")
    reads2b = torch.from_numpy(ga.pack(ps.reads)).to(dev)
    refs2b = torch.from_numpy(ga.pack(ps.refs)).to(dev)
    roff = torch.from_numpy(ps.read_off.astype(np.int64)).to(dev)
    foff = torch.from_numpy(ps.ref_off.astype(np.int64)).to(dev)
    for launch in (None, ga.make_launch(ga.FORM_PLAIN)):
        out, cigar = ctx.align_dev(reads2b, roff, refs2b, foff, ps.k, launch=launch)
        torch.cuda.synchronize()
        res = out.cpu().numpy().view(ga.RESULT_DTYPE).reshape(-1)
        elems = cigar.cpu().numpy().view(np.uint32)
        for i in range(ps.n_pairs):
            assert res["edit_distance"][i] == res_h["edit_distance"][i]
            o, n = int(res["cigar_off"][i]), int(res["cigar_len"][i])
            assert ga.decode_cigar(elems[o:o + n]) == cig_h[i]


def test_device_pack_matches_host_pack(ctx):
    import torch
    rng = np.random.default_rng(5)
    codes = rng.integers(0, 4, 100_003).astype(np.uint8)
    text = gen.to_ascii(codes)
    dev = torch.device("cuda:0")
    a = torch.frombuffer(bytearray(text), dtype=torch.uint8).to(dev)
    packed = torch.zeros((len(text) + 3) // 4, dtype=torch.uint8, device=dev)
    bad = torch.zeros(1, dtype=torch.int32, device=dev)
    ctx.pack_dev(a, packed, bad)
    torch.cuda.synchronize()
    assert int(bad.item()) == 0
    assert (packed.cpu().numpy() == ga.pack(text)).all()
    bad.zero_()
    a[7] = ord("N")
    ctx.pack_dev(a, packed, bad)
    torch.cuda.synchronize()
    assert int(bad.item()) == 1


@pytest.mark.parametrize("offset", [0, 1, 16])
@pytest.mark.parametrize("n", [0, 1, 15, 16, 17, 33, 4099])
def test_device_pack_sizes_alignment_and_case(ctx, offset, n):
    # the 16-bases-per-thread kernel (16-byte aligned input) and the byte path
    # (any other alignment), ragged tails, lower case and bytes outside ACGT
    import torch
    rng = np.random.default_rng(100 + n + offset)
    text = bytearray(gen.to_ascii(rng.integers(0, 4, n).astype(np.uint8)))
    for q in range(0, n, 5):
        text[q] = text[q] | 0x20  # lower case
    bad_at = [q for q in range(3, n, 37)]
    for q in bad_at:
        text[q] = ord("N") if q % 2 else ord("x")
    dev = torch.device("cuda:0")
    buf = torch.zeros(n + offset + 16, dtype=torch.uint8, device=dev)
    buf[offset:offset + n] = torch.frombuffer(bytearray(text) or bytearray(1), dtype=torch.uint8)[:n].to(dev)
    a = buf[offset:offset + n]
    packed = torch.full(((n + 3) // 4 + 4,), 0xEE, dtype=torch.uint8, device=dev)
    bad = torch.zeros(1, dtype=torch.int32, device=dev)
    ctx.pack_dev(a, packed[:(n + 3) // 4], bad)
    torch.cuda.synchronize()
    got = packed.cpu().numpy()
    assert int(bad.item()) == len(bad_at)
    # bytes outside ACGT are coded 0 (as A)
    fixed = bytearray(bytes(text).upper())
    for q in bad_at:
        fixed[q] = ord("A")
    assert (got[:(n + 3) // 4] == ga.pack(bytes(fixed))).all()
    assert (got[(n + 3) // 4:] == 0xEE).all()  # nothing written past the packed length


def test_alphabet_error_is_reported(ctx):
    with pytest.raises(ga.GenasmError) as e:
        ctx.align(["ACGT"], ["ACNT"], 5)
    assert e.value.code == ga.capi.E_ALPHABET


def _decode_dev(out, cigar, n):
    res = out.cpu().numpy().view(ga.RESULT_DTYPE).reshape(-1)[:n]
    elems = cigar.cpu().numpy().view(np.uint32)
    got = []
    for r in res:
        assert r["flags"] == 0
        o, k = int(r["cigar_off"]), int(r["cigar_len"])
        got.append((int(r["edit_distance"]), int(r["ref_begin"]), int(r["ref_end"]),
                    int(r["n_windows"]), ga.decode_cigar(elems[o:o + k])))
    return got


@pytest.mark.parametrize("form", sorted(FORMS))
def test_graph_capture_replays(ctx, form):
    # The device form captured in a HIP graph (through torch's capture of the
    # current stream): every replay, with eager work and synchronizations
    # between replays, rewrites the same results. The graph keeps using its
    # context's scratch, so it gets a context of its own.
    import torch
    ps = gen.make("uneven", 300, start=900)
    want = expected(ps)
    dev = torch.device("cuda:0")
    reads2b = torch.from_numpy(ga.pack(ps.reads)).to(dev)
    refs2b = torch.from_numpy(ga.pack(ps.refs)).to(dev)
    roff = torch.from_numpy(ps.read_off.astype(np.int64)).to(dev)
    foff = torch.from_numpy(ps.ref_off.astype(np.int64)).to(dev)
    nr, nf = int(ps.read_off[-1]), int(ps.ref_off[-1])
    out = torch.empty((ps.n_pairs, 32), dtype=torch.uint8, device=dev)
    cigar = torch.empty(nr + nf, dtype=torch.int32, device=dev)
    gctx = ga.Context(0)
    try:
        kw = dict(launch=FORMS[form], out=out, cigar=cigar, total_read_bases=nr,
                  total_ref_bases=nf)
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            gctx.align_dev(reads2b, roff, refs2b, foff, ps.k, **kw)  # sizes the scratch
        torch.cuda.synchronize()
        assert_same(ps, want, _decode_dev(out, cigar, ps.n_pairs), f"{form} eager")
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            gctx.align_dev(reads2b, roff, refs2b, foff, ps.k, **kw)
        small = gen.make("short100", 50)
        for rep in range(3):
            out.zero_()
            cigar.fill_(-1)
            torch.cuda.synchronize()
            on_gpu(ctx, small)  # eager work on another context between replays
            g.replay()
            torch.cuda.synchronize()
            assert_same(ps, want, _decode_dev(out, cigar, ps.n_pairs), f"{form} replay {rep}")
    finally:
        gctx.close()


@pytest.mark.parametrize("form,variant", [("batched", "improved"), ("compact", "improved"),
                                          ("plain", "improved"), ("unimproved", "uncompressed")])
def test_work_counters_match_oracle(ctx, form, variant):
    # The device work counters (profiling) against the oracle variant with the
    # same storage scheme: DC word operations, DP cells, stored table words and,
    # for the edge-word form, the words its traceback reads.
    ps = gen.make("uneven", 60, start=3000)
    res, _, _, _ = oracle.batch(ps, variant)
    assert (res["status"] == 0).all() and (res["score"] >= 0).all()
    ctx.profile(True)
    try:
        ctx.align([ps.read(i) for i in range(ps.n_pairs)], [ps.ref(i) for i in range(ps.n_pairs)],
                  ps.k, ps.W, ps.O, FORMS[form])
        pr = ctx.profile_read()
    finally:
        ctx.profile(False)
    assert pr["n_pairs"] == ps.n_pairs
    assert pr["window_cells"] == int(res["cells_window"].sum())
    assert pr["search_cells"] == int(res["cells_search"].sum())
    assert pr["window_word_ops"] == int(res["word_ops"].sum())
    assert pr["table_words"] == int(res["words_stored"].sum())
    assert pr["windows"] == int(res["n_windows"].sum())
    if variant == "uncompressed":
        assert pr["tb_reads"] == int(res["words_read"].sum())


def test_autotune_picks_caches_and_reloads(ctx, tmp_path):
    import torch
    ps = gen.make("uneven", 400, start=1200)
    want = expected(ps)
    dev = torch.device("cuda:0")
    r2 = torch.from_numpy(ga.pack(ps.reads)).to(dev)
    f2 = torch.from_numpy(ga.pack(ps.refs)).to(dev)
    ro = torch.from_numpy(ps.read_off.astype(np.int64)).to(dev)
    fo = torch.from_numpy(ps.ref_off.astype(np.int64)).to(dev)
    tctx = ga.Context(0)
    try:
        best, ms, out, cigar = tctx.autotune_dev(r2, ro, f2, fo, ps.k)
        torch.cuda.synchronize()
        assert ms > 0 and tctx.tune_cache_size() == 1
        assert best.form == ga.FORM_BATCHED
        assert_same(ps, want, _decode_dev(out, cigar, ps.n_pairs), "autotune runs")
        # a call without a launch takes the cached pick; results are unchanged
        out.zero_()
        tctx.align_dev(r2, ro, f2, fo, ps.k, out=out, cigar=cigar)
        torch.cuda.synchronize()
        assert_same(ps, want, _decode_dev(out, cigar, ps.n_pairs), "cached launch")
        path = str(tmp_path / "tune.txt")
        tctx.tune_cache_save(path)
        fields = [ln.split() for ln in open(path) if not ln.startswith("#")]
        assert len(fields) == 1 and int(fields[0][7]) == best.hard_row
        assert int(fields[0][9]) == best.tb_prefetch and int(fields[0][10]) == best.hard_share
        other = ga.Context(0)
        try:
            other.tune_cache_load(path)
            assert other.tune_cache_size() == 1
        finally:
            other.close()
    finally:
        tctx.close()


def test_captured_context_refuses_to_grow(ctx):
    # A call recorded into a graph pins the context: a later call that needs
    # larger buffers fails with GENASM_E_PINNED instead of freeing what the
    # graph uses, the graph keeps replaying correct results, and after
    # genasm_unpin (graph gone) the context grows again.
    import torch
    small = gen.make("uneven", 100, start=4000)
    big = gen.make("uneven", 2000, start=4000)
    dev = torch.device("cuda:0")

    def tensors(ps):
        return (torch.from_numpy(ga.pack(ps.reads)).to(dev), torch.from_numpy(ps.read_off.astype(np.int64)).to(dev),
                torch.from_numpy(ga.pack(ps.refs)).to(dev), torch.from_numpy(ps.ref_off.astype(np.int64)).to(dev))

    ts, tb = tensors(small), tensors(big)
    nr, nf = int(small.read_off[-1]), int(small.ref_off[-1])
    out = torch.empty((small.n_pairs, 32), dtype=torch.uint8, device=dev)
    cigar = torch.empty(nr + nf, dtype=torch.int32, device=dev)
    want = expected(small)
    gctx = ga.Context(0)
    try:
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            gctx.align_dev(*ts, small.k, out=out, cigar=cigar)  # sizes the buffers
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            # totals given: reading them from the offsets would copy to the host
            gctx.align_dev(*ts, small.k, out=out, cigar=cigar,
                           total_read_bases=nr - int(small.read_off[0]),
                           total_ref_bases=nf - int(small.ref_off[0]))
        with pytest.raises(ga.GenasmError) as e:
            gctx.align_dev(*tb, big.k)
        assert e.value.code == ga.capi.E_PINNED
        torch.cuda.synchronize()
        for rep in range(2):
            out.zero_()
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            assert_same(small, want, _decode_dev(out, cigar, small.n_pairs), f"pinned replay {rep}")
        del g
        torch.cuda.synchronize()
        gctx.unpin()
        bout, bcig = gctx.align_dev(*tb, big.k)
        torch.cuda.synchronize()
        assert_same(big, expected(big), _decode_dev(bout, bcig, big.n_pairs), "after unpin")
    finally:
        gctx.close()


def test_host_form_nospace_writes_nothing(ctx):
    # GENASM_E_NOSPACE reports the size needed and leaves the results untouched
    import ctypes
    ps = gen.make("short100", 20)
    r, roff = ga.capi._concat([ps.read(i) for i in range(ps.n_pairs)])
    f, foff = ga.capi._concat([ps.ref(i) for i in range(ps.n_pairs)])
    out = np.full(ps.n_pairs, 0x5A, dtype=np.uint8).repeat(32).view(ga.RESULT_DTYPE)
    before = out.copy()
    buf = np.full(8, 0x33, dtype=np.uint8)
    need = ctypes.c_uint64(0)
    u64p = ctypes.POINTER(ctypes.c_uint64)
    rc = ga.capi.lib().genasm_batch_align(ctx._ctx, r, roff.ctypes.data_as(u64p), f,
                                          foff.ctypes.data_as(u64p), ps.n_pairs, ps.k, ps.W, ps.O,
                                          out.ctypes.data, buf.ctypes.data, len(buf),
                                          ctypes.byref(need), None)
    assert rc == ga.capi.E_NOSPACE
    assert need.value > len(buf)
    assert out.tobytes() == before.tobytes() and (buf == 0x33).all()
    # with the reported size the call succeeds and matches the oracle
    buf = np.zeros(need.value, dtype=np.uint8)
    rc = ga.capi.lib().genasm_batch_align(ctx._ctx, r, roff.ctypes.data_as(u64p), f,
                                          foff.ctypes.data_as(u64p), ps.n_pairs, ps.k, ps.W, ps.O,
                                          out.ctypes.data, buf.ctypes.data, len(buf),
                                          ctypes.byref(need), None)
    assert rc == 0
    text = buf.tobytes()
    got = [(int(x["edit_distance"]), int(x["ref_begin"]), int(x["ref_end"]), int(x["n_windows"]),
            text[int(x["cigar_off"]):int(x["cigar_off"]) + int(x["cigar_len"])].decode()) for x in out]
    assert_same(ps, expected(ps), got, "after E_NOSPACE")


def test_injected_allocation_failure(monkeypatch):
    # With GENASM_FAIL_ALLOC=1 every device allocation fails: a fresh context's
    # first device-form call and a server's creation return GENASM_E_NOMEM,
    # nothing is launched, and the same context works once the variable is gone.
    import torch
    ps = gen.make("short100", 50, start=70)
    want = expected(ps)
    fresh = ga.Context(0)
    try:
        monkeypatch.setenv("GENASM_FAIL_ALLOC", "1")
        with pytest.raises(ga.GenasmError) as e:
            on_gpu(fresh, ps)
        assert e.value.code == ga.capi.E_NOMEM
        with pytest.raises(ga.GenasmError) as e:
            ga.Server(fresh, ps.k, ps.W, ps.O)
        assert e.value.code == ga.capi.E_NOMEM
        monkeypatch.delenv("GENASM_FAIL_ALLOC")
        torch.cuda.synchronize()
        assert_same(ps, want, on_gpu(fresh, ps), "after the injected failure")
    finally:
        fresh.close()


def test_measured_peaks_are_plausible(ctx):
    """genasm_measure_peaks: every rate positive and each microbenchmark
    within what one MI355X can do (below the published or derived peaks; the
    64-bit shift, the funnel shift and the DPP move each issuing at about half
    the rate of a plain int32 operation: their instruction rates stay well
    below the int32 rate, the shift counting two operations per instruction)."""
    pk = ctx.measure_peaks()
    assert pk["compute_units"] == 256
    for key in ("dc_mix_tops", "int32_tops", "shift64_tops", "funnel_tops", "dpp_tops"):
        assert 1.0 < pk[key] < 2 * 78.6, (key, pk[key])
    for key, ops_per_instruction in (("shift64_tops", 2), ("funnel_tops", 1), ("dpp_tops", 1)):
        assert pk[key] / ops_per_instruction <= 0.6 * pk["int32_tops"], (key, pk[key], pk["int32_tops"])
    assert 0.5 < pk["hbm_tbps"] < 8.0
    assert pk["lds_tbps"] > 1.0


@pytest.mark.parametrize("W,O", [(64, 24), (64, 56), (32, 20), (48, 8)])
@pytest.mark.parametrize("hard_lanes", [16, 32])
def test_deep_windows_across_overlaps(ctx, W, O, hard_lanes):
    # 1,000-base prefixes of decoy and true pairs: the decoys' windows need
    # three or more DC passes, so the boundary row between passes, the spilled
    # passes and their traceback reads all run; W - O below and above the width
    # where every lane of a group takes part in the boundary-row store
    ps = gen.make("long10k", 8, start=4)
    cut = gen.from_lists("deep", [ps.read(i)[:1000] for i in range(ps.n_pairs)],
                         [ps.ref(i)[:1100] for i in range(ps.n_pairs)], 64, W, O)
    assert ps.decoy.any()
    L = ga.make_launch(ga.FORM_BATCHED, hard_lanes=hard_lanes, table_bits=64)
    assert_same(cut, expected(cut), on_gpu(ctx, cut, L), f"deep W={W} O={O} hard_lanes={hard_lanes}")
