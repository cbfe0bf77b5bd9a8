#!/usr/bin/env python3
"""Benchmark of the GenASM hot path on one MI355X.

One step = the whole path over one batch already resident in device memory:
2-bit packing of the ASCII reads and references, the start search, and the
windowed DC + traceback with run-length CIGAR output (batched form: search
kernels, then the persistent window kernel with its work queue). Prints ONE
JSON line on stdout; progress goes to stderr.

Default workload: 20,000 pairs of 10 kb reads with 10% PacBio-like edits,
reference = true segment +-500 bp, 30% unrelated 10 kb decoys, k=64, W=64,
O=24 (synthetic, seeded).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# int32 VALU peak of MI355X: 256 CUs x 128 lanes per cycle (4 SIMDs, a wave64
# 32-bit operation issued in two passes of 32 lanes) x 2.4 GHz = 78.6 T
# operations/s, the rate behind the published 157.3 TFLOP/s fp32 vector peak
# (one fused multiply-add counted as two flops).
INT32_PEAK_TOPS = 256 * 128 * 2.4e9 / 1e12

# HBM traffic of the window kernel, from rocprofv3 FETCH_SIZE / WRITE_SIZE runs
# scaled by a copy kernel of known size; valid only for the kernel source it was
# measured on.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_windows_long10k_traffic.json")
KERNEL_SRC = os.path.join(ROOT, "paper_2203_15561_amd", "csrc", "kernels.hip")


def measured_traffic(workload: str):
    import hashlib
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
        with open(KERNEL_SRC, "rb") as f:
            src_hash = hashlib.sha256(f.read()).hexdigest()
    except (OSError, ValueError):
        return None
    if rec.get("kernels_sha256") != src_hash or rec.get("workload") != workload:
        return None  # the kernel changed since the counters were taken
    return rec


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def rle(ops: str) -> str:
    out, k = [], 0
    while k < len(ops):
        j = k
        while j < len(ops) and ops[j] == ops[k]:
            j += 1
        out.append(f"{j - k}{ops[k]}")
        k = j
    return "".join(out)


def measured_peaks(ctx, achieved):
    """The device limits measured by the library's microbenchmarks, and the
    window kernel's rate against the recurrence's own instruction mix."""
    pk = ctx.measure_peaks()
    return {"dc_mix_tops": pk["dc_mix_tops"], "int32_tops": pk["int32_tops"],
            "lds_tbps": pk["lds_tbps"], "hbm_tbps": pk["hbm_tbps"],
            "shift64_tops": pk["shift64_tops"], "funnel_tops": pk["funnel_tops"],
            "dpp_tops": pk["dpp_tops"],
            "frac_of_dc_mix": achieved / pk["dc_mix_tops"],
            "frac_of_int32": achieved / pk["int32_tops"]}


def provenance(gen, dev):
    """Source revision, device architecture and workload seeds of the run."""
    import torch
    try:
        with open(os.path.join(ROOT, "paper_2203_15561_amd", "BUILD_INFO.json")) as f:
            info = json.load(f)
    except (OSError, ValueError):
        info = {}
    props = torch.cuda.get_device_properties(dev)
    return {"git": info.get("git"), "git_dirty": info.get("git_dirty"), "device": props.name,
            "arch": getattr(props, "gcnArchName", None), "compute_units": props.multi_processor_count,
            "seeds": {name: w[0] for name, w in gen.WORKLOADS.items()}}


def serving_leg(ga, gen, ctx, args):
    """Serving form on the request mix (70% 150 bp at 1%, 30% 1-30 kb at 10%).

    The same requests are first aligned as one batch through the device form
    in the plain and the batched launch: that gives the cells of the mix (the
    library's work counters) and the two launches' GCUPS. A saturated run then
    queues every request at once through the server (pre-packed bases,
    genasm_submit_batch; completions through genasm_poll_batch) and checks
    every completion against the batched form's result, CIGAR included.
    Open-loop runs with Poisson arrivals at a sweep of rates up to the
    saturated rate give latency percentiles, from each request's scheduled
    arrival to the time its CIGAR reached host memory."""
    import torch
    t0 = time.time()
    pool = gen.make("serving", args.serving_requests)
    n = pool.n_pairs
    r2, f2 = ga.pack(pool.reads), ga.pack(pool.refs)
    roff, foff = pool.read_off.astype(np.uint64), pool.ref_off.astype(np.uint64)
    short = np.diff(pool.read_off) <= 1000
    log(f"serving: {n} requests generated in {time.time() - t0:.1f} s")
    out = {"mix": gen.DESCRIPTIONS["serving"], "requests": n, "k": pool.k, "W": pool.W, "O": pool.O}

    # the mix as one batch: cells, plain and batched launches
    dev = torch.device("cuda:0")
    d_r2, d_f2 = torch.from_numpy(r2).to(dev), torch.from_numpy(f2).to(dev)
    d_ro = torch.from_numpy(roff.astype(np.int64)).to(dev)
    d_fo = torch.from_numpy(foff.astype(np.int64)).to(dev)
    best, _, b_out, b_cig = ctx.autotune_dev(d_r2, d_ro, d_f2, d_fo, pool.k, pool.W, pool.O)
    ctx.profile(True)
    ctx.align_dev(d_r2, d_ro, d_f2, d_fo, pool.k, pool.W, pool.O, launch=best, out=b_out, cigar=b_cig)
    pr = ctx.profile_read()
    ctx.profile(False)
    cells = pr["window_cells"] + pr["search_cells"]
    ref_res = b_out.cpu().numpy().view(ga.RESULT_DTYPE).reshape(-1)[:n].copy()
    ref_el = b_cig.cpu().numpy().view(np.uint32)
    for form, L in (("batched_launch", best), ("plain_launch", ga.make_launch(ga.FORM_PLAIN))):
        ctx.align_dev(d_r2, d_ro, d_f2, d_fo, pool.k, pool.W, pool.O, launch=L, out=b_out, cigar=b_cig)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(2):
            ctx.align_dev(d_r2, d_ro, d_f2, d_fo, pool.k, pool.W, pool.O, launch=L, out=b_out,
                          cigar=b_cig)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 2
        out[form] = {"ms": ms, "requests_per_s": n / (ms / 1e3), "gcups": cells / (ms / 1e3) / 1e9}
        log(f"serving mix as one batch, {form}: {ms:.2f} ms ({out[form]['gcups']:.0f} GCUPS)")
    out["cells"] = int(cells)
    del d_r2, d_f2, d_ro, d_fo, b_out, b_cig

    def submit_range(srv, lo, hi, tags):
        rc, acc = srv.submit_batch(r2, roff[lo:hi + 1], f2, foff[lo:hi + 1], tags[lo:hi])
        assert rc in (0, ga.capi.E_BUSY), rc
        return acc

    def collect(srv, infos, runs, timeout_ms):
        info, el = srv.poll_arrays(timeout_ms=timeout_ms)
        if len(info):
            infos.append(info)
            runs.append(el)
        return len(info)

    with ga.Server(ctx, pool.k, pool.W, pool.O, cigar_runs=1, max_pending=n + 1) as srv:
        tags = np.arange(n, dtype=np.uint64)
        # warm-up: the first 2,000 requests
        w = min(2000, n)
        submit_range(srv, 0, w, tags)
        got = 0
        while got < w:
            got += len(srv.poll_arrays(timeout_ms=20)[0])
        # saturated: every request queued at once
        st0 = srv.stats()
        infos, runs = [], []
        t_start = ga.now_ns()
        i = 0
        while i < n:
            i += submit_range(srv, i, min(n, i + 8192), tags)
            collect(srv, infos, runs, 0)
        t_submitted = ga.now_ns()
        done = sum(len(x) for x in infos)
        t_log = time.time() + 10
        while done < n:
            done += collect(srv, infos, runs, 20)
            if time.time() > t_log:
                log(f"serving: {done} of {n} requests completed")
                t_log = time.time() + 10
        st1 = srv.stats()
        info = np.concatenate(infos)
        t_end = int(info["done_ns"].max())
        secs = (t_end - t_start) / 1e9
        iters = st1["iterations"] - st0["iterations"]
        # every completion equals the batched form's result, CIGAR included
        order = np.argsort(info["tag"])
        info = info[order]
        assert (info["tag"] == tags).all()
        res = info["result"]
        assert (res["flags"] == 0).all()
        for f in ("edit_distance", "ref_begin", "ref_end", "n_windows", "cigar_len"):
            assert (res[f] == ref_res[f]).all(), f
        el = np.concatenate(runs)
        # completion elements were appended in arrival order; rebuild per-tag offsets
        starts = np.concatenate(([0], np.cumsum([len(x) for x in runs])))[:-1]
        base = np.concatenate([np.full(len(x), s0, np.int64) for x, s0 in zip(infos, starts)])[order]
        off = base + res["cigar_off"].astype(np.int64)
        ln = res["cigar_len"].astype(np.int64)
        idx = np.repeat(off - np.concatenate(([0], np.cumsum(ln)))[:-1], ln) + np.arange(ln.sum())
        ref_idx = np.repeat(ref_res["cigar_off"].astype(np.int64) - np.concatenate(([0], np.cumsum(ln)))[:-1],
                            ln) + np.arange(ln.sum())
        assert np.array_equal(el[idx], ref_el[ref_idx]), "serving CIGARs differ from the batched form"
        sat = n / secs
        out["saturated"] = {
            "requests": n, "seconds": secs, "requests_per_s": sat, "gcups": cells / secs / 1e9,
            "submit_seconds": (t_submitted - t_start) / 1e9,
            "iterations": iters, "device_ms": st1["device_ms"] - st0["device_ms"],
            "device_busy": (st1["device_ms"] - st0["device_ms"]) / 1e3 / secs,
            "over_plain_launch": (cells / secs / 1e9) / out["plain_launch"]["gcups"],
            "over_batched_launch": (cells / secs / 1e9) / out["batched_launch"]["gcups"],
            "checked": "every completion equals the batched device form (result fields and CIGAR)"}
        log(f"serving saturated: {sat:.0f} req/s ({out['saturated']['gcups']:.0f} GCUPS) over {n} "
            f"requests, {iters} iterations; plain launch {out['plain_launch']['gcups']:.0f} GCUPS")

        # open loop: Poisson arrivals at each rate, submitted at their scheduled times
        rates = [float(x) for x in args.serving_rates.split(",") if x.strip()]
        rates = sorted({r for r in rates if r < 0.95 * sat} | {0.5 * sat, 0.8 * sat})
        out["open_loop"] = []
        for k_rate, rate in enumerate(rates):
            n_open = int(min(n, max(2000, rate * args.serving_seconds)))
            rng = np.random.default_rng(2203 + k_rate)
            sched_rel = np.cumsum(rng.exponential(1.0 / rate, n_open) * 1e9).astype(np.int64)
            infos, runs = [], []
            t_begin = ga.now_ns() + 1_000_000
            sched = t_begin + sched_rel
            i = 0
            while i < n_open:
                now = ga.now_ns()
                j = int(np.searchsorted(sched, now, side="right"))
                if j > i:
                    i += submit_range(srv, i, j, tags)
                collect(srv, infos, runs, 0)
                if i < n_open:
                    wait = (sched[i] - ga.now_ns()) / 1e9
                    if wait > 0.0002:
                        time.sleep(min(wait, 0.001))
            done = sum(len(x) for x in infos)
            t_end_wait = time.time() + 300
            while done < n_open:
                assert time.time() < t_end_wait, "open-loop requests did not complete"
                done += collect(srv, infos, runs, 20)
            info = np.concatenate(infos)
            info = info[np.argsort(info["tag"])]
            assert (info["result"]["flags"] == 0).all()
            assert (info["result"]["edit_distance"] == ref_res["edit_distance"][:n_open]).all()
            lat = (info["done_ns"].astype(np.int64) - sched) / 1e6
            sh = short[:n_open]
            pct = lambda a, q: float(np.percentile(a, q)) if len(a) else None
            o = {"arrival_rate_per_s": rate, "requests": n_open,
                 "completed_per_s": n_open / ((int(info["done_ns"].max()) - t_begin) / 1e9),
                 "p50_ms": pct(lat, 50), "p99_ms": pct(lat, 99), "mean_ms": float(lat.mean()),
                 "short_p50_ms": pct(lat[sh], 50), "short_p99_ms": pct(lat[sh], 99),
                 "long_p50_ms": pct(lat[~sh], 50), "long_p99_ms": pct(lat[~sh], 99)}
            out["open_loop"].append(o)
            log(f"serving open loop at {rate:.0f} req/s: p50 {o['p50_ms']:.2f} ms, p99 "
                f"{o['p99_ms']:.2f} ms (150 bp: p50 {o['short_p50_ms']:.2f} / p99 "
                f"{o['short_p99_ms']:.2f} ms)")
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="long10k")
    ap.add_argument("--pairs", type=int, default=None, help="pairs (default: the full workload)")
    ap.add_argument("--no-plain", action="store_true", help="skip timing the plain form")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=20000,
                    help="pairs of the workload the CPU oracle aligns for the baseline")
    ap.add_argument("--verify", type=int, default=32, help="pairs checked against the oracle")
    ap.add_argument("--group-lanes", type=int, default=0)
    ap.add_argument("--lds-rows", type=int, default=0)
    ap.add_argument("--workers-per-cu", type=int, default=0)
    ap.add_argument("--hard-row", type=int, default=0)
    ap.add_argument("--hard-lanes", type=int, default=0)
    ap.add_argument("--hard-share", type=int, default=-1)
    ap.add_argument("--table-bits", type=int, default=0)
    ap.add_argument("--search-per-cu", type=int, default=0)
    ap.add_argument("--no-autotune", action="store_true",
                    help="time the default launch instead of the autotuner's pick")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving leg")
    ap.add_argument("--copy-calibration-mb", type=int, default=0,
                    help="after the timed region, run one plain device copy of this many MiB "
                         "(reference kernel for scaling HBM byte counters)")
    ap.add_argument("--serving-requests", type=int, default=40000,
                    help="requests of the serving mix (saturated run; the open-loop runs use "
                         "its first requests)")
    ap.add_argument("--serving-seconds", type=float, default=2.0,
                    help="length of each open-loop arrival schedule")
    ap.add_argument("--serving-rates", default="1000,3000,10000,30000,100000,300000,1000000",
                    help="open-loop arrival rates (req/s), comma-separated; those above the "
                         "saturated rate are skipped, and 50%% and 80%% of it are added")
    ap.add_argument("--serving-only", action="store_true",
                    help="run only the serving leg (for profiling it)")
    ap.add_argument("--no-graph", action="store_true", help="skip timing the graph-captured step")
    ap.add_argument("--no-filter", action="store_true", help="skip the pre-alignment filter leg")
    ap.add_argument("--no-other-configs", action="store_true",
                    help="skip the batched-vs-plain legs on the 100 bp, 250 bp and uneven workloads")
    ap.add_argument("--filter-pairs", type=int, default=20000,
                    help="pairs of the 250 bp workload for the filter leg")
    ap.add_argument("--no-unimproved", action="store_true",
                    help="skip the ablation run without the three improvements")
    ap.add_argument("--no-end-to-end", action="store_true", help="skip the host-memory form timing")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: pairs are independent and this build runs on a single "
              "MI355X; run it with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2203_15561_amd as ga
    from workloads import gen

    if args.serving_only:
        ctx = ga.Context(0)
        print(json.dumps({"serving": serving_leg(ga, gen, ctx, args)}), flush=True)
        ctx.close()
        return

    t0 = time.time()
    ps = gen.make(args.workload, args.pairs)
    log(f"generated {ps.n_pairs} pairs of {args.workload} in {time.time() - t0:.1f}s")
    dev = torch.device("cuda:0")
    reads_ascii = torch.from_numpy(np.frombuffer(gen.to_ascii(ps.reads), dtype=np.uint8).copy()).to(dev)
    refs_ascii = torch.from_numpy(np.frombuffer(gen.to_ascii(ps.refs), dtype=np.uint8).copy()).to(dev)
    roff = torch.from_numpy(ps.read_off.astype(np.int64)).to(dev)
    foff = torch.from_numpy(ps.ref_off.astype(np.int64)).to(dev)
    nr, nf = int(ps.read_off[-1]), int(ps.ref_off[-1])
    reads2b = torch.empty((nr + 3) // 4, dtype=torch.uint8, device=dev)
    refs2b = torch.empty((nf + 3) // 4, dtype=torch.uint8, device=dev)
    bad = torch.zeros(1, dtype=torch.int32, device=dev)
    out = torch.empty((ps.n_pairs, 32), dtype=torch.uint8, device=dev)
    cigar = torch.empty(nr + nf, dtype=torch.int32, device=dev)

    ctx = ga.Context(0)
    kw = {}
    if args.group_lanes:
        kw["group_lanes"] = args.group_lanes
    if args.lds_rows:
        kw["lds_rows"] = args.lds_rows
    if args.workers_per_cu:
        kw["workers_per_cu"] = args.workers_per_cu
    if args.hard_row:
        kw["hard_row"] = args.hard_row
    if args.hard_lanes:
        kw["hard_lanes"] = args.hard_lanes
    if args.hard_share >= 0:
        kw["hard_share"] = args.hard_share
    if args.table_bits:
        kw["table_bits"] = args.table_bits
    if args.search_per_cu:
        kw["search_per_cu"] = args.search_per_cu
    batched = ga.make_launch(ga.FORM_BATCHED, **kw)
    plain = ga.make_launch(ga.FORM_PLAIN)

    def step(launch):
        ctx.pack_dev(reads_ascii, reads2b, bad)
        ctx.pack_dev(refs_ascii, refs2b, bad)
        ctx.align_dev(reads2b, roff, refs2b, foff, ps.k, ps.W, ps.O, launch=launch, out=out,
                      cigar=cigar, total_read_bases=nr, total_ref_bases=nf)

    # warm-up
    for _ in range(args.warmup):
        step(batched)
    torch.cuda.synchronize()
    assert int(bad.item()) == 0
    log("warm-up done")
    tuned = None
    if not args.no_autotune and not kw:
        # the library's autotuner times its candidate launches on this batch
        t0 = time.time()
        batched, tms, _, _ = ctx.autotune_dev(reads2b, roff, refs2b, foff, ps.k, ps.W, ps.O,
                                              out=out, cigar=cigar, reps=2, total_read_bases=nr,
                                              total_ref_bases=nf)
        tuned = {"tuner_seconds": time.time() - t0, "best_ms": tms}
        log(f"autotune: table_bits {batched.table_bits}, hard_row {batched.hard_row}, hard_lanes "
            f"{batched.hard_lanes}, hard_share {batched.hard_share}, lds_rows "
            f"{batched.lds_rows}, workers_per_cu {batched.workers_per_cu}, search_lanes "
            f"{batched.search_lanes} ({tms:.2f} ms) in {tuned['tuner_seconds']:.1f} s")

    # work counters of one step (a profiled run), then the timed region: K steps
    # with stage times only (HIP events around each stage on the kernels' stream;
    # the kernels run as unprofiled), one profile read per step
    ctx.profile(1)
    step(batched)
    prc = ctx.profile_read()
    ctx.profile(2)
    win_ms, search_ms, total_ms = [], [], []
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(args.steps):
        step(batched)
        pr = ctx.profile_read()
        win_ms.append(pr["windows_ms"])
        search_ms.append(pr["search_ms"])
        total_ms.append(pr["total_ms"])
    ev1.record()
    torch.cuda.synchronize()
    ms_step = ev0.elapsed_time(ev1) / args.steps
    ctx.profile(False)
    log(f"batched: {ms_step:.2f} ms/step; window kernel {np.mean(win_ms):.2f} ms, search "
        f"{np.mean(search_ms):.2f} ms")

    res = out.cpu().numpy().view(ga.RESULT_DTYPE).reshape(-1)
    assert (res["flags"] == 0).all()

    if args.copy_calibration_mb:
        # one elementwise kernel that reads and writes exactly this many bytes
        nbytes = args.copy_calibration_mb << 20
        src = torch.ones(nbytes // 4, dtype=torch.int32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        torch.add(src, 1, out=dst)
        torch.cuda.synchronize()
        log(f"copy calibration: read {nbytes} B, wrote {nbytes} B")
        del src, dst

    # spot-check results against the oracle
    verified = 0
    if args.verify:
        import oracle
        idx = np.linspace(0, ps.n_pairs - 1, min(args.verify, ps.n_pairs)).astype(int)
        sub = ps.subset(idx)
        ro, ops, _, _ = oracle.batch(sub)
        elems = cigar.cpu().numpy().view(np.uint32)
        for j, i in enumerate(idx):
            r = res[i]
            o, n = int(r["cigar_off"]), int(r["cigar_len"])
            assert int(r["edit_distance"]) == int(ro["score"][j]), (i, r, ro[j])
            want = rle(oracle.pair_ops(sub, ro, ops, j)) if ro["score"][j] >= 0 else ""
            assert ga.decode_cigar(elems[o:o + n]) == want, i
            verified += 1
        log(f"verified {verified} pairs against the oracle")

    pr = {**prc, **{k: v for k, v in pr.items() if k.endswith("_ms")}}
    cells = pr["window_cells"] + pr["search_cells"]
    int_ops_windows = 2 * pr["window_word_ops"]  # two 32-bit halves per 64-bit word op
    achieved = int_ops_windows / (np.mean(win_ms) / 1e3) / 1e12
    line = {
        "metric": "alignments/s (10 kb reads, 10% edits, batched form)",
        "value": ps.n_pairs / (ms_step / 1e3),
        "unit": "alignments/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {gen.DESCRIPTIONS[args.workload]}",
                   "pairs": ps.n_pairs, "k": ps.k, "W": ps.W, "O": ps.O, "form": "batched",
                   "group_lanes": batched.group_lanes, "lds_rows": batched.lds_rows,
                   "workers_per_cu": batched.workers_per_cu, "hard_row": batched.hard_row,
                   "hard_share": batched.hard_share,
                   "hard_lanes": batched.hard_lanes, "search_lanes": batched.search_lanes,
                   "table_bits": batched.table_bits, "search_per_cu": batched.search_per_cu,
                   "autotuned": tuned is not None},
        "autotune": tuned,
        "gcups": cells / (ms_step / 1e3) / 1e9,
        "window_kernel_ms": float(np.mean(win_ms)),
        "search_ms": float(np.mean(search_ms)),
        "roofline": {"bound": "alu", "kernel": "k_windows (window DC + traceback)",
                     "achieved": achieved, "peak": INT32_PEAK_TOPS, "unit": "TOP/s",
                     "frac": achieved / INT32_PEAK_TOPS, "traffic": None,
                     "ops_per_launch": int_ops_windows,
                     "peak_basis": "256 CUs x 128 int32 lanes per cycle x 2.4 GHz",
                     "measured": measured_peaks(ctx, achieved)},
        "work": {k: int(v) for k, v in pr.items() if not k.endswith("_ms")},
        "verified_pairs": verified,
        "provenance": provenance(gen, dev),
    }

    traffic = measured_traffic(args.workload) if ps.n_pairs == 20000 else None
    if traffic:
        line["roofline"]["traffic"] = traffic["hbm_bytes_per_launch"]
        line["roofline"]["traffic_detail"] = {k: traffic[k] for k in
                                              ("fetch_bytes", "write_bytes", "fetch_scale",
                                               "write_scale", "source")}

    if not args.no_plain:
        torch.cuda.synchronize()
        step(plain)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        step(plain)
        e1.record()
        torch.cuda.synchronize()
        pm = e0.elapsed_time(e1)
        line["plain"] = {"alignments_per_s": ps.n_pairs / (pm / 1e3), "ms": pm,
                         "gcups": cells / (pm / 1e3) / 1e9}
        log(f"plain: {pm:.2f} ms/step")

    if not args.no_unimproved:
        # ablation: the same step with the unimproved window (every row, four
        # edge words per entry in device memory); a profiled run gives its work
        # counters, an unprofiled one its time
        unimp = ga.make_launch(ga.FORM_UNIMPROVED)
        ctx.profile(True)
        step(unimp)
        pu = ctx.profile_read()
        ctx.profile(False)
        torch.cuda.synchronize()
        u0, u1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        u0.record()
        step(unimp)
        u1.record()
        torch.cuda.synchronize()
        um = u0.elapsed_time(u1)
        res_u = out.cpu().numpy().view(ga.RESULT_DTYPE).reshape(-1)
        assert (res_u["edit_distance"] == res["edit_distance"]).all()
        win = max(pr["windows"], 1)
        line["unimproved"] = {
            "alignments_per_s": ps.n_pairs / (um / 1e3), "ms": um,
            "table_words": int(pu["table_words"]), "tb_reads": int(pu["tb_reads"]),
            "window_word_ops": int(pu["window_word_ops"])}
        line["improvements"] = {
            "speedup_batched_over_unimproved": um / ms_step,
            "speedup_plain_over_unimproved": um / line["plain"]["ms"] if "plain" in line else None,
            "table_words_per_window": {"improved": pr["table_words"] / win,
                                       "unimproved": pu["table_words"] / max(pu["windows"], 1)},
            "footprint_reduction": (pu["table_words"] / max(pu["windows"], 1)) / (pr["table_words"] / win),
            "access_reduction": (pu["table_words"] + pu["tb_reads"]) / (pr["table_words"] + pr["tb_reads"]),
            "dc_work_reduction": pu["window_word_ops"] / max(pr["window_word_ops"], 1),
            "paper": {"footprint_reduction": 24, "access_reduction": 12, "gpu_speedup": 5.9},
        }
        log(f"unimproved: {um:.1f} ms/step ({um / ms_step:.1f}x the batched step); footprint "
            f"{line['improvements']['footprint_reduction']:.1f}x, accesses "
            f"{line['improvements']['access_reduction']:.1f}x smaller with the improvements")

    if not args.no_graph:
        # the same step captured once in a HIP graph (through torch's stream
        # capture) and replayed; a context of its own keeps the captured scratch
        gctx = ga.Context(0)
        gs = torch.cuda.Stream()
        gs.wait_stream(torch.cuda.current_stream())

        def gstep():
            gctx.pack_dev(reads_ascii, reads2b, bad)
            gctx.pack_dev(refs_ascii, refs2b, bad)
            gctx.align_dev(reads2b, roff, refs2b, foff, ps.k, ps.W, ps.O, launch=batched, out=out,
                           cigar=cigar, total_read_bases=nr, total_ref_bases=nf)

        with torch.cuda.stream(gs):
            gstep()
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph, stream=gs):
            gstep()
        graph.replay()
        torch.cuda.synchronize()
        g0, g1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        g0.record()
        for _ in range(args.steps):
            graph.replay()
        g1.record()
        torch.cuda.synchronize()
        gms = g0.elapsed_time(g1) / args.steps
        res_g = out.cpu().numpy().view(ga.RESULT_DTYPE).reshape(-1)
        assert (res_g["edit_distance"] == res["edit_distance"]).all()
        line["graph"] = {"alignments_per_s": ps.n_pairs / (gms / 1e3), "ms_per_step": gms}
        log(f"graph replay: {gms:.2f} ms/step")
        del graph
        gctx.close()

    if not args.no_end_to_end:
        # host memory in and out: ASCII upload, packing, the whole path, CIGAR text back
        r_ascii, f_ascii = gen.to_ascii(ps.reads), gen.to_ascii(ps.refs)
        ctx.align_buffers(r_ascii, ps.read_off, f_ascii, ps.ref_off, ps.k, ps.W, ps.O, batched)
        t0 = time.perf_counter()
        res_h, _ = ctx.align_buffers(r_ascii, ps.read_off, f_ascii, ps.ref_off, ps.k, ps.W, ps.O,
                                     batched)
        e2e = time.perf_counter() - t0
        assert (res_h["edit_distance"] == res["edit_distance"]).all()
        line["end_to_end"] = {"alignments_per_s": ps.n_pairs / e2e, "seconds": e2e,
                              "what": "host ASCII in, CIGAR text out (PCIe and host gather included)"}
        log(f"end to end (host form): {e2e * 1e3:.1f} ms")

    if not args.no_filter:
        # score-only mode on 250 bp reads (2% edits, 20 bp flanks), k = 15
        fps = gen.make("short250", args.filter_pairs)
        fr2 = torch.from_numpy(ga.pack(fps.reads)).to(dev)
        ff2 = torch.from_numpy(ga.pack(fps.refs)).to(dev)
        fro = torch.from_numpy(fps.read_off.astype(np.int64)).to(dev)
        ffo = torch.from_numpy(fps.ref_off.astype(np.int64)).to(dev)
        fmax = int(np.diff(fps.read_off).max())
        dist, start = ctx.filter_dev(fr2, fro, ff2, ffo, fps.k, fmax)
        torch.cuda.synchronize()
        f0, f1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        f0.record()
        for _ in range(args.steps):
            ctx.filter_dev(fr2, fro, ff2, ffo, fps.k, fmax, dist=dist, start=start)
        f1.record()
        torch.cuda.synchronize()
        fms = f0.elapsed_time(f1) / args.steps
        cells = float((np.diff(fps.read_off) * np.diff(fps.ref_off)).sum())
        line["filter"] = {"workload": f"short250: {fps.n_pairs} pairs, k={fps.k}",
                          "pairs_per_s": fps.n_pairs / (fms / 1e3), "ms": fms,
                          "gcups": cells / (fms / 1e3) / 1e9,
                          "accepted": float((dist.cpu().numpy() >= 0).mean())}
        log(f"filter: {fms:.3f} ms for {fps.n_pairs} pairs ({line['filter']['gcups']:.0f} GCUPS)")

    if not args.no_other_configs:
        # the other batch workloads: batched (autotuned) against the plain launch
        line["other_configs"] = {}
        for wname in ("short100", "short250", "uneven"):
            ops = gen.make(wname)
            o_r2 = torch.from_numpy(ga.pack(ops.reads)).to(dev)
            o_f2 = torch.from_numpy(ga.pack(ops.refs)).to(dev)
            o_ro = torch.from_numpy(ops.read_off.astype(np.int64)).to(dev)
            o_fo = torch.from_numpy(ops.ref_off.astype(np.int64)).to(dev)
            o_best, _, o_out, o_cig = ctx.autotune_dev(o_r2, o_ro, o_f2, o_fo, ops.k, ops.W, ops.O)
            o_cells = None
            res_o = {}
            for form, L in (("batched", o_best), ("plain", ga.make_launch(ga.FORM_PLAIN))):
                ctx.align_dev(o_r2, o_ro, o_f2, o_fo, ops.k, ops.W, ops.O, launch=L, out=o_out,
                              cigar=o_cig)
                torch.cuda.synchronize()
                ctx.profile(True)
                ctx.align_dev(o_r2, o_ro, o_f2, o_fo, ops.k, ops.W, ops.O, launch=L, out=o_out,
                              cigar=o_cig)
                pr_o = ctx.profile_read()
                ctx.profile(False)
                o0, o1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                o0.record()
                for _ in range(args.steps):
                    ctx.align_dev(o_r2, o_ro, o_f2, o_fo, ops.k, ops.W, ops.O, launch=L, out=o_out,
                                  cigar=o_cig)
                o1.record()
                torch.cuda.synchronize()
                oms = o0.elapsed_time(o1) / args.steps
                o_cells = pr_o["window_cells"] + pr_o["search_cells"]
                res_o[form] = {"ms": oms, "alignments_per_s": ops.n_pairs / (oms / 1e3),
                               "gcups": o_cells / (oms / 1e3) / 1e9}
                res_o[form + "_scores"] = o_out.cpu().numpy().view(ga.RESULT_DTYPE)["edit_distance"].copy()
            # the batched form captured once in a HIP graph (a context of its own
            # keeps the captured scratch) and replayed
            gctx = ga.Context(0)
            gs = torch.cuda.Stream()
            gs.wait_stream(torch.cuda.current_stream())
            nr_o = int(ops.read_off[-1] - ops.read_off[0])
            nf_o = int(ops.ref_off[-1] - ops.ref_off[0])

            def ocall():
                gctx.align_dev(o_r2, o_ro, o_f2, o_fo, ops.k, ops.W, ops.O, launch=o_best, out=o_out,
                               cigar=o_cig, total_read_bases=nr_o, total_ref_bases=nf_o)

            with torch.cuda.stream(gs):
                ocall()
            torch.cuda.synchronize()
            og = torch.cuda.CUDAGraph()
            with torch.cuda.graph(og, stream=gs):
                ocall()
            og.replay()
            torch.cuda.synchronize()
            o0, o1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            o0.record()
            for _ in range(args.steps):
                og.replay()
            o1.record()
            torch.cuda.synchronize()
            gms = o0.elapsed_time(o1) / args.steps
            res_g = o_out.cpu().numpy().view(ga.RESULT_DTYPE)["edit_distance"].copy()
            assert (res_g == res_o["plain_scores"]).all()
            res_o["batched_graph"] = {"ms": gms, "alignments_per_s": ops.n_pairs / (gms / 1e3),
                                      "gcups": o_cells / (gms / 1e3) / 1e9}
            del og
            gctx.close()
            assert (res_o["batched_scores"] == res_o["plain_scores"]).all()
            del res_o["batched_scores"], res_o["plain_scores"]
            res_o["pairs"] = ops.n_pairs
            res_o["workload"] = gen.DESCRIPTIONS[wname]
            res_o["batched_over_plain"] = res_o["plain"]["ms"] / res_o["batched"]["ms"]
            line["other_configs"][wname] = res_o
            log(f"{wname}: batched {res_o['batched']['ms']:.2f} ms, plain {res_o['plain']['ms']:.2f} ms "
                f"({res_o['batched_over_plain']:.2f}x)")
            del o_r2, o_f2, o_ro, o_fo, o_out, o_cig

    if not args.no_serving:
        line["serving"] = serving_leg(ga, gen, ctx, args)

    if not args.no_cpu_baseline:
        import oracle
        sample = min(args.cpu_sample, ps.n_pairs)
        sub = ps if sample == ps.n_pairs else ps.subset(np.arange(sample))
        _, _, secs, used = oracle.batch(sub)
        one = ps.subset(np.arange(min(500, ps.n_pairs)))
        _, _, secs1, _ = oracle.batch(one, nthreads=1)
        unc = ps.subset(np.arange(min(300, ps.n_pairs)))
        _, _, secs_u, used_u = oracle.batch(unc, "uncompressed")
        line["cpu_baseline"] = {
            "value": sample / secs, "unit": "alignments/s", "cores": used, "kind": "oracle",
            "sample": f"first {sample} pairs of {args.workload} (same mix), improved form, "
                      f"{used} threads, {secs:.2f} s wall",
            "per_core": {"alignments_per_s": one.n_pairs / secs1, "pairs": one.n_pairs},
            "uncompressed": {"alignments_per_s": unc.n_pairs / secs_u, "pairs": unc.n_pairs,
                             "cores": used_u}}
        log(f"cpu oracle: {sample / secs:.1f} alignments/s on {used} threads; "
            f"{one.n_pairs / secs1:.1f} on 1 thread; uncompressed {unc.n_pairs / secs_u:.1f} "
            f"on {used_u} threads")

    ctx.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
