"""GPU parity at full size: every pair of every batch workload (short100:
1,000 pairs; short250: 100,000; long10k: 20,000; uneven: 50,000) through the
C ABI, compared with the CPU oracle pair by pair on edit distance, reference
span, window count and every CIGAR run. The bar is bit-exact (integer work).

Launches: the batched form with its default launch, with compact groups and
with the autotuner's pick, the plain form, the unimproved form (long10k), a persistent grid so
small that every window group takes many pairs in turn (its LDS header, spill
area and run state carried from one pair to the next), and the host-memory
form (short250), whose CIGAR text is compared run by run."""
import numpy as np
import pytest

import oracle
import paper_2203_15561_amd as ga
from tests._helpers import assert_batch_matches, device_run_elements, text_run_elements
from workloads import gen

pytestmark = pytest.mark.gpu

_CACHE = {}


def workload(name, n=None):
    """(pairs, oracle results, oracle ops, device tensors) of a workload; one
    workload is kept at a time (the long ones take gigabytes)."""
    key = (name, n)
    if key not in _CACHE:
        import torch
        _CACHE.clear()
        ps = gen.make(name, n)
        ores, oops, _, _ = oracle.batch(ps)
        dev = torch.device("cuda:0")
        t = dict(r2=torch.from_numpy(ga.pack(ps.reads)).to(dev),
                 f2=torch.from_numpy(ga.pack(ps.refs)).to(dev),
                 ro=torch.from_numpy(ps.read_off.astype(np.int64)).to(dev),
                 fo=torch.from_numpy(ps.ref_off.astype(np.int64)).to(dev))
        print(f"[full-size] {name}: {ps.n_pairs} pairs, {ps.total_bases()} bases", flush=True)
        _CACHE[key] = (ps, ores, oops, t)
    return _CACHE[key]


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    c = ga.Context(0)
    yield c
    c.close()


def run_dev(ctx, name, launch, n=None, label=""):
    import torch
    ps, ores, oops, t = workload(name, n)
    print(f"[full-size] {label or name}: launching", flush=True)
    out, cig = ctx.align_dev(t["r2"], t["ro"], t["f2"], t["fo"], ps.k, ps.W, ps.O, launch=launch)
    torch.cuda.synchronize()
    gres = out.cpu().numpy().view(ga.RESULT_DTYPE).reshape(-1)[:ps.n_pairs]
    el = cig.cpu().numpy().view(np.uint32)
    assert_batch_matches(ps, ores, oops, gres,
                         lambda lo, hi: device_run_elements(gres, el, lo, hi), label or name)
    return ps, gres


BATCH_WORKLOADS = ["short100", "short250", "long10k", "uneven"]


@pytest.mark.parametrize("name", BATCH_WORKLOADS)
def test_batched_default_every_pair(ctx, name):
    run_dev(ctx, name, ga.make_launch(ga.FORM_BATCHED), label=f"{name}/batched default")


@pytest.mark.parametrize("name", BATCH_WORKLOADS)
def test_batched_autotuned_every_pair(ctx, name):
    import torch
    ps, _, _, t = workload(name)
    tctx = ga.Context(0)
    try:
        best, ms, _, _ = tctx.autotune_dev(t["r2"], t["ro"], t["f2"], t["fo"], ps.k, ps.W, ps.O)
        torch.cuda.synchronize()
        print(f"[full-size] {name}: tuner pick hard_row {best.hard_row} hard_lanes {best.hard_lanes}"
              f" lds_rows {best.lds_rows} workers {best.workers_per_cu} ({ms:.2f} ms)", flush=True)
        # the pick, explicitly, and a call without a launch (the cached pick)
        run_dev(tctx, name, best, label=f"{name}/batched autotuned")
        run_dev(tctx, name, None, label=f"{name}/batched cached pick")
    finally:
        tctx.close()


@pytest.mark.parametrize("name", BATCH_WORKLOADS)
def test_compact_every_pair(ctx, name):
    run_dev(ctx, name, ga.make_launch(ga.FORM_BATCHED, table_bits=32), label=f"{name}/compact")


@pytest.mark.parametrize("name", BATCH_WORKLOADS)
def test_plain_every_pair(ctx, name):
    run_dev(ctx, name, ga.make_launch(ga.FORM_PLAIN), label=f"{name}/plain")


def test_unimproved_long10k_every_pair(ctx):
    run_dev(ctx, "long10k", ga.make_launch(ga.FORM_UNIMPROVED), label="long10k/unimproved")


@pytest.mark.parametrize("variant", [dict(), dict(hard_lanes=32), dict(hard_lanes=64),
                                     dict(hard_row=65), dict(hard_row=-1, hard_lanes=32),
                                     dict(table_bits=32), dict(table_bits=32, hard_row=65)])
def test_groups_take_many_pairs(ctx, variant):
    # 5,000 long pairs on one workgroup per compute unit: every 16-lane group
    # (or 32-/64-lane hard group) runs several pairs in turn
    run_dev(ctx, "long10k", ga.make_launch(ga.FORM_BATCHED, workers_per_cu=1, **variant), n=5000,
            label=f"long10k[:5000]/one worker per CU {variant}")


def test_host_form_short250_every_pair(ctx):
    ps, ores, oops, _ = workload("short250")
    r_ascii, f_ascii = gen.to_ascii(ps.reads), gen.to_ascii(ps.refs)
    print("[full-size] short250 host form: launching", flush=True)
    gres, text = ctx.align_buffers(r_ascii, ps.read_off, f_ascii, ps.ref_off, ps.k, ps.W, ps.O)
    assert_batch_matches(ps, ores, oops, gres, lambda lo, hi: text_run_elements(gres, text, lo, hi),
                         "short250/host form")
