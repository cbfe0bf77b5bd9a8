"""Seeded synthetic (read, reference) pair generator.

This module only draws random sequences and applies random edits. It holds
none of the alignment arithmetic, so both the CPU oracle and the GPU path can
take their inputs from it.

Bases are coded A=0, C=1, G=2, T=3 (uint8). Every pair has its own generator,
seeded from ``SeedSequence([seed, pair_index])``, so the pair a test sees
does not depend on how many pairs were generated alongside it.

The workloads stand in for the paper's evaluation set (Results section:
simulated 10 kb PacBio reads from the human genome, aligned at every
candidate location a read mapper reports, decoy locations included). Neither
the genome nor the simulator is available, so bases are i.i.d. uniform and
the error model is the per-event mutation model below.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

ASCII = np.frombuffer(b"ACGT", dtype=np.uint8)

# Event kinds of the mutation model.
SUB, INS, DEL = 0, 1, 2


@dataclass
class PairSet:
    """Concatenated pairs: pair i is reads[read_off[i]:read_off[i+1]] against
    refs[ref_off[i]:ref_off[i+1]]."""

    name: str
    reads: np.ndarray  # uint8 codes 0..3
    read_off: np.ndarray  # uint64, n_pairs + 1
    refs: np.ndarray
    ref_off: np.ndarray
    k: int
    W: int = 64
    O: int = 24
    decoy: np.ndarray | None = None  # bool per pair, where the workload has decoys
    meta: dict = field(default_factory=dict)

    @property
    def n_pairs(self) -> int:
        return len(self.read_off) - 1

    def read(self, i: int) -> np.ndarray:
        return self.reads[self.read_off[i]:self.read_off[i + 1]]

    def ref(self, i: int) -> np.ndarray:
        return self.refs[self.ref_off[i]:self.ref_off[i + 1]]

    def subset(self, idx) -> "PairSet":
        idx = np.asarray(idx, dtype=np.int64)
        reads = [self.read(int(i)) for i in idx]
        refs = [self.ref(int(i)) for i in idx]
        ps = from_lists(self.name + "[subset]", reads, refs, self.k, self.W, self.O)
        if self.decoy is not None:
            ps.decoy = self.decoy[idx]
        ps.meta = dict(self.meta)
        return ps

    def total_bases(self) -> int:
        return int(self.read_off[-1] + self.ref_off[-1])


def from_lists(name, reads, refs, k, W=64, O=24) -> PairSet:
    """Build a PairSet from lists of code arrays (or ACGT strings)."""
    reads = [_as_codes(r) for r in reads]
    refs = [_as_codes(r) for r in refs]
    read_off = np.zeros(len(reads) + 1, dtype=np.uint64)
    ref_off = np.zeros(len(refs) + 1, dtype=np.uint64)
    read_off[1:] = np.cumsum([len(r) for r in reads], dtype=np.uint64)
    ref_off[1:] = np.cumsum([len(r) for r in refs], dtype=np.uint64)
    cat = lambda xs: (np.concatenate(xs).astype(np.uint8) if xs else np.zeros(0, np.uint8))
    return PairSet(name, cat(reads), read_off, cat(refs), ref_off, k, W, O)


def _as_codes(s) -> np.ndarray:
    if isinstance(s, (bytes, str)):
        b = s.encode() if isinstance(s, str) else s
        lut = np.full(256, 255, dtype=np.uint8)
        for code, ch in enumerate(b"ACGT"):
            lut[ch] = code
            lut[ch + 32] = code
        out = lut[np.frombuffer(b, dtype=np.uint8)]
        if (out == 255).any():
            raise ValueError("sequence holds a byte outside ACGTacgt")
        return out
    return np.asarray(s, dtype=np.uint8)


def to_ascii(codes: np.ndarray) -> bytes:
    return ASCII[np.asarray(codes, dtype=np.uint8)].tobytes()


def pair_rng(seed: int, idx: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([seed, idx]))


def random_bases(rng: np.random.Generator, n: int) -> np.ndarray:
    return rng.integers(0, 4, size=n, dtype=np.uint8)


def mutate(rng: np.random.Generator, src: np.ndarray, rate: float, mix, geom_p=None) -> np.ndarray:
    """Apply E = round(rate * |src| / mu) edit events to ``src``.

    ``mix`` = probabilities of (substitution, insertion, deletion). Event
    lengths are 1 for substitutions; for insertions and deletions they are 1
    when ``geom_p`` is None, else Geometric(geom_p) on {1, 2, ...}. ``mu`` is
    the mean event length under that mix. Events sit at distinct uniform
    positions of ``src``. An insertion puts its random bases before its
    position; a substitution replaces the base with one of the other three,
    uniformly; a deletion removes src[pos:pos+len], clipped so that it stops
    at the next event's position and at the end of ``src``.
    """
    n = len(src)
    mix = np.asarray(mix, dtype=np.float64)
    mix = mix / mix.sum()
    mean_indel = 1.0 if geom_p is None else 1.0 / geom_p
    mu = mix[SUB] + (mix[INS] + mix[DEL]) * mean_indel
    n_ev = int(round(rate * n / mu))
    n_ev = min(n_ev, n)
    if n_ev == 0 or n == 0:
        return src.copy()
    pos = np.sort(rng.choice(n, size=n_ev, replace=False)).astype(np.int64)
    kind = rng.choice(3, size=n_ev, p=mix)
    if geom_p is None:
        length = np.ones(n_ev, dtype=np.int64)
    else:
        length = rng.geometric(geom_p, size=n_ev).astype(np.int64)
    length[kind == SUB] = 1
    nxt = np.append(pos[1:], n)
    dlen = np.where(kind == DEL, np.minimum(length, nxt - pos), 0)

    keep = np.ones(n, dtype=bool)
    keep[pos[kind == SUB]] = False
    if dlen.any():
        starts = pos[dlen > 0]
        lens = dlen[dlen > 0]
        idx = np.repeat(starts, lens) + (np.arange(lens.sum()) - np.repeat(np.cumsum(lens) - lens, lens))
        keep[idx] = False

    # inserted bases: substitutions contribute one new base at their position,
    # insertions contribute `length` random bases before their position.
    sub_pos = pos[kind == SUB]
    sub_new = ((src[sub_pos].astype(np.int64) + rng.integers(1, 4, size=len(sub_pos))) % 4).astype(np.uint8)
    ins_sel = kind == INS
    ins_pos = np.repeat(pos[ins_sel], length[ins_sel])
    ins_new = random_bases(rng, len(ins_pos))

    new_pos = np.concatenate([sub_pos, ins_pos])
    new_val = np.concatenate([sub_new, ins_new])
    kept_idx = np.nonzero(keep)[0]
    # order key: a new base placed before source index q sorts as 2q, the kept
    # source base q as 2q + 1; the stable sort keeps insertion order.
    keys = np.concatenate([2 * new_pos, 2 * kept_idx + 1])
    vals = np.concatenate([new_val, src[kept_idx]])
    order = np.argsort(keys, kind="stable")
    return vals[order].astype(np.uint8)


# Workload definitions -------------------------------------------------------

PACBIO_MIX = (0.15, 0.50, 0.35)  # substitution, insertion, deletion
PACBIO_GEOM_P = 0.7


def _c1_pair(rng):
    read = random_bases(rng, 100)
    core = mutate(rng, read, 0.05, (1 / 3, 1 / 3, 1 / 3))
    ref = np.concatenate([random_bases(rng, 10), core, random_bases(rng, 10)])
    return read, ref, False


def _c2_pair(rng):
    read = random_bases(rng, 250)
    core = mutate(rng, read, 0.02, (0.90, 0.05, 0.05))
    ref = np.concatenate([random_bases(rng, 20), core, random_bases(rng, 20)])
    return read, ref, False


def _c3_pair(rng):
    seg = random_bases(rng, 10_000)
    read = mutate(rng, seg, 0.10, PACBIO_MIX, PACBIO_GEOM_P)
    decoy = bool(rng.random() < 0.3)
    if decoy:
        ref = random_bases(rng, 10_000)
    else:
        ref = np.concatenate([random_bases(rng, 500), seg, random_bases(rng, 500)])
    return read, ref, decoy


def _c4_pair(rng):
    L = int(round(np.exp(rng.normal(np.log(2000.0), 1.0))))
    L = min(max(L, 100), 30_000)
    e = rng.uniform(0.01, 0.15)
    seg = random_bases(rng, L)
    read = mutate(rng, seg, e, PACBIO_MIX, PACBIO_GEOM_P)
    ref = np.concatenate([random_bases(rng, 50), seg, random_bases(rng, 50)])
    return read, ref, False


def serving_request(rng):
    """One request of the serving mix: 70% short (150 bp, 1% error, 20 bp
    flanks), 30% long (1-30 kb, 10% PacBio-like error, 500 bp flanks)."""
    if rng.random() < 0.7:
        seg = random_bases(rng, 150)
        read = mutate(rng, seg, 0.01, (0.90, 0.05, 0.05))
        ref = np.concatenate([random_bases(rng, 20), seg, random_bases(rng, 20)])
    else:
        L = int(rng.integers(1_000, 30_001))
        seg = random_bases(rng, L)
        read = mutate(rng, seg, 0.10, PACBIO_MIX, PACBIO_GEOM_P)
        ref = np.concatenate([random_bases(rng, 500), seg, random_bases(rng, 500)])
    return read, ref, False


WORKLOADS = {
    # name: (seed, pair fn, default pair count, k)
    "short100": (101, _c1_pair, 1_000, 10),
    "short250": (102, _c2_pair, 100_000, 15),
    "long10k": (103, _c3_pair, 20_000, 64),
    "uneven": (104, _c4_pair, 50_000, 64),
    "serving": (105, serving_request, 200_000, 64),
}

DESCRIPTIONS = {
    "short100": "1,000 pairs: 100 bp reads, reference = read with 5% S/I/D edits + 10 bp flanks, k=10",
    "short250": "100,000 pairs: 250 bp reads, 2% edits (90% S, 5% I, 5% D) + 20 bp flanks, k=15",
    "long10k": "20,000 pairs: 10 kb reads, 10% PacBio-like edits, reference = segment +-500 bp, 30% unrelated 10 kb decoys, k=64",
    "uneven": "50,000 pairs: log-normal lengths (median 2 kb, 100 bp-30 kb), 1-15% edits, 50 bp flanks, k=64",
    "serving": "request mix: 70% 150 bp at 1%, 30% 1-30 kb at 10%",
}


def make(name: str, n_pairs: int | None = None, start: int = 0) -> PairSet:
    """Generate pairs start .. start+n_pairs-1 of workload ``name``."""
    seed, fn, default_n, k = WORKLOADS[name]
    if n_pairs is None:
        n_pairs = default_n - start
    reads, refs, decoys = [], [], []
    for i in range(start, start + n_pairs):
        r, t, dec = fn(pair_rng(seed, i))
        reads.append(r)
        refs.append(t)
        decoys.append(dec)
    ps = from_lists(name, reads, refs, k)
    ps.decoy = np.asarray(decoys, dtype=bool)
    ps.meta = {"seed": seed, "start": start, "description": DESCRIPTIONS[name]}
    return ps


def fuzz(seed: int, n_pairs: int, max_len: int = 300, related: float = 0.7) -> list:
    """Random pairs for property tests: lengths 0..max_len, error rates
    0-40%, a mix of related and unrelated references."""
    out = []
    for i in range(n_pairs):
        rng = pair_rng(seed, i)
        m = int(rng.integers(0, max_len + 1))
        read = random_bases(rng, m)
        if rng.random() < related and m > 0:
            e = rng.uniform(0.0, 0.4)
            core = mutate(rng, read, e, (1 / 3, 1 / 3, 1 / 3),
                          None if rng.random() < 0.5 else PACBIO_GEOM_P)
            fl = int(rng.integers(0, 30))
            fr = int(rng.integers(0, 30))
            ref = np.concatenate([random_bases(rng, fl), core, random_bases(rng, fr)])
        else:
            ref = random_bases(rng, int(rng.integers(0, max_len + 1)))
        out.append((read, ref))
    return out
