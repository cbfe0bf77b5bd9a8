"""The GENASM_DEBUG build on the GPU: its invariant checks (window bounds,
LDS and spill rows of every pass, CIGAR runs per window) and its queue audit
(every queued pair taken by exactly one window worker) hold on a mixed
workload in each launch form, and its results match the oracle's. It runs in
a child process because the library variant is chosen when the binding
loads."""
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import numpy as np
import oracle
import paper_2203_15561_amd as ga
from paper_2203_15561_amd import capi
from tests._helpers import rle
from workloads import gen

assert capi.LIB_PATH.endswith("libgenasm_debug.so"), capi.LIB_PATH
ctx = ga.Context(0)
sets = [gen.make("short100", 300, start=11), gen.make("short250", 120, start=5),
        gen.make("long10k", 6, start=2)]
fuzz = gen.fuzz(2024, 40, max_len=300)
sets.append(gen.from_lists("fuzz", [p[0] for p in fuzz], [p[1] for p in fuzz], 7, 16, 8))
forms = {"batched": None, "plain": ga.make_launch(ga.FORM_PLAIN),
         "compact": ga.make_launch(ga.FORM_BATCHED, table_bits=32),
         "hard32": ga.make_launch(ga.FORM_BATCHED, hard_lanes=32, table_bits=64)}
for ps in sets:
    res, ops, _, _ = oracle.batch(ps)
    want = [(int(res["score"][i]), int(res["ref_begin"][i]) if res["score"][i] >= 0 else 0,
             int(res["ref_end"][i]) if res["score"][i] >= 0 else 0, int(res["n_windows"][i]),
             rle(oracle.pair_ops(ps, res, ops, i)) if res["score"][i] >= 0 else "")
            for i in range(ps.n_pairs)]
    reads = [ps.read(i) for i in range(ps.n_pairs)]
    refs = [ps.ref(i) for i in range(ps.n_pairs)]
    for name, launch in forms.items():
        print(f"debug build: {ps.name} {ps.n_pairs} pairs, {name}", flush=True)
        out, cig = ctx.align(reads, refs, ps.k, ps.W, ps.O, launch)
        flagged = np.nonzero(out["flags"])[0]
        assert flagged.size == 0, (ps.name, name, flagged[:10], out["flags"][flagged[:10]])
        got = [(int(r["edit_distance"]), int(r["ref_begin"]), int(r["ref_end"]),
                int(r["n_windows"]), c) for r, c in zip(out, cig)]
        bad = [i for i in range(ps.n_pairs) if got[i] != want[i]]
        assert not bad, (ps.name, name, bad[:5])
ctx.close()
print("debug build: all clean", flush=True)
"""


def test_debug_build_checks_hold_and_results_match():
    env = dict(os.environ, GENASM_LIB_VARIANT="debug")
    r = subprocess.run([sys.executable, "-u", "-c", CHILD], cwd=ROOT, env=env, timeout=300,
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "all clean" in r.stdout
