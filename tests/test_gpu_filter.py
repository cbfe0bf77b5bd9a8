"""GPU tests of the pre-alignment filter (score-only mode) through the C ABI:
distance and leftmost start of the best reference substring for the whole
read, or rejection above k, bit-exact against the oracle's definition."""
import numpy as np
import pytest

import oracle
import paper_2203_15561_amd as ga
from workloads import gen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    c = ga.Context(0)
    yield c
    c.close()


def check(ctx, reads, refs, k, label):
    dist, start = ctx.filter(reads, refs, k)
    bad = []
    for i, (r, t) in enumerate(zip(reads, refs)):
        want = oracle.filter_pair(r, t, k)
        got = (int(dist[i]), int(start[i]) if dist[i] >= 0 else 0)
        if got != want:
            bad.append((i, want, got))
    assert not bad, f"{label}: {len(bad)} of {len(reads)} differ, first {bad[0]}"
    return dist


@pytest.mark.parametrize("name,n,k", [("short100", 1000, 10), ("short250", 2000, 15)])
def test_filter_short_read_workloads(ctx, name, n, k):
    ps = gen.make(name, n)
    reads = [ps.read(i) for i in range(ps.n_pairs)]
    refs = [ps.ref(i) for i in range(ps.n_pairs)]
    dist = check(ctx, reads, refs, k, name)
    assert (dist >= 0).mean() > 0.5  # most true pairs pass the filter


@pytest.mark.parametrize("k", [0, 7, 63])
def test_filter_lengths_up_to_1024(ctx, k):
    # every row width (1, 2, 4, 8 and 16 words) and degenerate pairs
    pairs = gen.fuzz(8080 + k, 160, max_len=1024)
    pairs += [("", ""), ("", "ACGT"), ("ACGT", ""), ("A" * 64, "A" * 64), ("A" * 65, "C" * 65),
              ("ACGT" * 256, "ACGT" * 256), ("T" * 1024, "")]
    check(ctx, [p[0] for p in pairs], [p[1] for p in pairs], k, f"fuzz k={k}")


def test_filter_device_form_matches_host_form(ctx):
    import torch
    ps = gen.make("short250", 500, start=7000)
    reads = [ps.read(i) for i in range(ps.n_pairs)]
    refs = [ps.ref(i) for i in range(ps.n_pairs)]
    dist_h, start_h = ctx.filter(reads, refs, 15)
    dev = torch.device("cuda:0")
    r2 = torch.from_numpy(ga.pack(ps.reads)).to(dev)
    f2 = torch.from_numpy(ga.pack(ps.refs)).to(dev)
    ro = torch.from_numpy(ps.read_off.astype(np.int64)).to(dev)
    fo = torch.from_numpy(ps.ref_off.astype(np.int64)).to(dev)
    dist, start = ctx.filter_dev(r2, ro, f2, fo, 15, int(np.diff(ps.read_off).max()))
    torch.cuda.synchronize()
    assert (dist.cpu().numpy() == dist_h).all()
    assert (start.cpu().numpy().view(np.uint32) == start_h).all()


def test_filter_argument_errors(ctx):
    with pytest.raises(ga.GenasmError) as e:
        ctx.filter(["ACGT"], ["ACGT"], 64)
    assert e.value.code == ga.capi.E_INVAL
    with pytest.raises(ga.GenasmError) as e:
        ctx.filter(["A" * 1025], ["A" * 1025], 5)
    assert e.value.code == ga.capi.E_TOOLONG
    with pytest.raises(ga.GenasmError) as e:
        ctx.filter(["ACGN"], ["ACGT"], 5)
    assert e.value.code == ga.capi.E_ALPHABET
