"""The no-allocation device form (genasm_batch_align_dev_noalloc) through the
C ABI, against the allocating device form (genasm_batch_align_dev) on the same
inputs: every result field and every CIGAR element equal, bit for bit, on two
calls in a row, the second on a smaller batch, so that it runs over what the
first left in the shared static scratch; plain and batched forms, and both
checked against the CPU oracle as well. Also: a graph-captured
no-allocation call replayed with other no-allocation calls between the
replays, a batch too large for the static scratch (an error, nothing
written), and the unimproved form (refused)."""
import ctypes

import numpy as np
import pytest

import oracle
import paper_2203_15561_amd as ga
from tests._helpers import assert_batch_matches, device_run_elements
from workloads import gen

pytestmark = pytest.mark.gpu

FORMS = {"batched": ga.make_launch(ga.FORM_BATCHED), "plain": ga.make_launch(ga.FORM_PLAIN)}


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    c = ga.Context(0)
    yield c
    c.close()


def device_batch(ps):
    import torch
    dev = torch.device("cuda:0")
    return dict(r2=torch.from_numpy(ga.pack(ps.reads)).to(dev),
                f2=torch.from_numpy(ga.pack(ps.refs)).to(dev),
                ro=torch.from_numpy(ps.read_off.astype(np.int64)).to(dev),
                fo=torch.from_numpy(ps.ref_off.astype(np.int64)).to(dev),
                nr=int(ps.read_off[-1] - ps.read_off[0]), nf=int(ps.ref_off[-1] - ps.ref_off[0]))


def outputs(ps, t):
    """Result and CIGAR buffers of a batch, filled with a sentinel."""
    import torch
    out = torch.full((ps.n_pairs, 32), 0xA5, dtype=torch.uint8, device=t["ro"].device)
    cig = torch.full((t["nr"] + t["nf"],), -1, dtype=torch.int32, device=t["ro"].device)
    return out, cig


def call(ctx, ps, t, launch, noalloc, out, cig, stream=None):
    print(f"[noalloc] {'no-allocation' if noalloc else 'allocating'} call: {ps.n_pairs} pairs, "
          f"{t['nr'] + t['nf']} bases, form {launch.form}", flush=True)
    ctx.align_dev(t["r2"], t["ro"], t["f2"], t["fo"], ps.k, ps.W, ps.O, launch=launch, out=out,
                  cigar=cig, stream=stream, total_read_bases=t["nr"], total_ref_bases=t["nf"],
                  noalloc=noalloc)


def host(out, cig, n):
    import torch
    torch.cuda.synchronize()
    res = out.cpu().numpy().view(ga.RESULT_DTYPE).reshape(-1)[:n].copy()
    return res, cig.cpu().numpy().view(np.uint32).copy()


def assert_equal_outputs(ps, a, b, label):
    (ra, ea), (rb, eb) = a, b
    for f in ga.RESULT_DTYPE.names:
        bad = np.flatnonzero(ra[f] != rb[f])
        assert not len(bad), f"{label}: field {f} differs on {len(bad)} pairs, first {bad[:5]}"
    for lo in range(0, ps.n_pairs, 2000):
        hi = min(ps.n_pairs, lo + 2000)
        xa, ca = device_run_elements(ra, ea, lo, hi)
        xb, cb = device_run_elements(rb, eb, lo, hi)
        assert np.array_equal(ca, cb) and np.array_equal(xa, xb), f"{label}: CIGARs differ in {lo}..{hi}"


@pytest.mark.parametrize("form", sorted(FORMS))
def test_noalloc_matches_allocating_form(ctx, form):
    launch = FORMS[form]
    # the second batch is smaller (fewer pairs and bases) than the first
    first = gen.make("uneven", 3000, start=7000)
    second = gen.make("long10k", 300, start=9000)
    assert second.n_pairs < first.n_pairs and second.total_bases() < first.total_bases()
    for ps in (first, second):
        t = device_batch(ps)
        ores, oops, _, _ = oracle.batch(ps)
        o1, c1 = outputs(ps, t)
        call(ctx, ps, t, launch, True, o1, c1)
        got = host(o1, c1, ps.n_pairs)
        o2, c2 = outputs(ps, t)
        call(ctx, ps, t, launch, False, o2, c2)
        ref = host(o2, c2, ps.n_pairs)
        assert_equal_outputs(ps, got, ref, f"{form} no-allocation vs allocating, {ps.n_pairs} pairs")
        assert_batch_matches(ps, ores, oops, got[0],
                             lambda lo, hi: device_run_elements(got[0], got[1], lo, hi),
                             f"{form} no-allocation vs oracle, {ps.n_pairs} pairs")


def test_noalloc_graph_replays(ctx):
    # a captured no-allocation call, replayed three times; between the replays
    # an eager no-allocation call on another batch overwrites the static scratch
    import torch
    ps = gen.make("short250", 2000, start=50_000)
    other = gen.make("uneven", 200, start=12_000)
    t, t2 = device_batch(ps), device_batch(other)
    launch = FORMS["batched"]
    want_o, want_c = outputs(ps, t)
    call(ctx, ps, t, launch, False, want_o, want_c)
    want = host(want_o, want_c, ps.n_pairs)
    ores2, oops2, _, _ = oracle.batch(other)
    out, cig = outputs(ps, t)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    print("[noalloc] capturing a no-allocation call", flush=True)
    with torch.cuda.graph(g, stream=s):
        call(ctx, ps, t, launch, True, out, cig, stream=s.cuda_stream)
    torch.cuda.synchronize()
    for rep in range(3):
        out.fill_(0xA5)
        cig.fill_(-1)
        torch.cuda.synchronize()
        print(f"[noalloc] replay {rep}", flush=True)
        g.replay()
        got = host(out, cig, ps.n_pairs)
        assert_equal_outputs(ps, got, want, f"graph replay {rep}")
        o2, c2 = outputs(other, t2)
        call(ctx, other, t2, launch, True, o2, c2)
        r2 = host(o2, c2, other.n_pairs)
        assert_batch_matches(other, ores2, oops2, r2[0],
                             lambda lo, hi: device_run_elements(r2[0], r2[1], lo, hi),
                             f"eager no-allocation call after replay {rep}")
    del g
    torch.cuda.synchronize()


def test_noalloc_batch_too_large(ctx):
    # 2 x 300 M bases: the bit planes alone need 150 MB, more than the static
    # scratch; the call returns GENASM_E_SCRATCH before launching anything
    import torch
    dev = torch.device("cuda:0")
    m = 300_000_000
    r2 = torch.zeros(m // 4, dtype=torch.uint8, device=dev)
    off = torch.tensor([0, m], dtype=torch.int64, device=dev)
    out = torch.full((1, 32), 0xA5, dtype=torch.uint8, device=dev)
    cig = torch.full((2 * m,), -1, dtype=torch.int32, device=dev)
    for form in sorted(FORMS):
        print(f"[noalloc] oversize batch, {form} form", flush=True)
        rc = ga.lib().genasm_batch_align_dev_noalloc(
            ctx._ctx, r2.data_ptr(), off.data_ptr(), r2.data_ptr(), off.data_ptr(), 1, m, m, 64,
            64, 24, out.data_ptr(), cig.data_ptr(), cig.numel(), ctypes.byref(FORMS[form]), None)
        assert rc == ga.capi.E_SCRATCH, rc
        assert str(ga.capi.NOALLOC_SCRATCH_BYTES) in ctx.last_error(), ctx.last_error()
    torch.cuda.synchronize()
    assert bool((out == 0xA5).all()) and bool((cig[:4096] == -1).all())


def test_noalloc_refuses_unimproved(ctx):
    import torch
    ps = gen.make("short100", 10)
    t = device_batch(ps)
    out, cig = outputs(ps, t)
    with pytest.raises(ga.GenasmError) as e:
        call(ctx, ps, t, ga.make_launch(ga.FORM_UNIMPROVED), True, out, cig)
    assert e.value.code == ga.capi.E_INVAL
    torch.cuda.synchronize()
