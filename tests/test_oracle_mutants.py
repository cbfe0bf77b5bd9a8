"""Planted mistakes: each mutant is a copy of the oracle source with one
plausible error (a dropped term, a wrong index, a wrong shift, a reversed
scan, a wrong stop rule, a miscounted score). The pin tests must reject every
mutant; a mutant that passes them all means the pins have a blind spot."""
import ctypes
import os
import tempfile

import pytest

import oracle
from tests import test_oracle_pins as pins

MUTANTS = {
    "drop_insertion_term": ("return match & substitution & insertion & deletion;",
                            "return match & substitution & deletion;"),
    "drop_deletion_term": ("return match & substitution & insertion & deletion;",
                           "return match & substitution & insertion;"),
    "substitution_unshifted": ("uint64_t substitution = r_up_right << 1;",
                               "uint64_t substitution = r_up_right;"),
    "insertion_wrong_column": ("uint64_t insertion = r_up_here << 1;",
                               "uint64_t insertion = r_up_right << 1;"),
    "all_ones_initial_column": ("return d >= 64 ? 0 : (~0ull << d);", "return ~0ull;"),
    "pattern_mask_reversed": ("pm[Pw[mw - 1 - q]] &= ~(1ull << q);", "pm[Pw[q]] &= ~(1ull << q);"),
    "rightmost_start": ("if (!(cur[i] & msb)) { found = d; *col = i; break; }",
                        "if (!(cur[i] & msb)) { found = d; *col = i; }"),
    "tb_insertion_reads_wrong_column": ("if ((*status = improved_read(c, d - 1, i, &w))) return 0;",
                                        "if ((*status = improved_read(c, d - 1, i + 1, &w))) return 0;"),
    "window_stop_one_late": ("while (p >= 0 && i < L && j < L) {",
                             "while (p >= 0 && i <= L && j < L) {"),
    "edits_miscounted": ("w.edits = dstar - d;", "w.edits = dstar;"),
    "sellers_free_read_start": ("cur[0] = r;", "cur[0] = 0;"),
    "sellers_mismatch_free": ("int64_t diag = prev[j - 1] + (P[r - 1] != T[j - 1]);",
                              "int64_t diag = prev[j - 1];"),
    "check_cigar_allows_x_on_equal": ("if (P[pi] == T[ti]) return -4;", ""),
    "filter_rightmost_start": ("if (prev[e] <= best) { best = prev[e]; best_e = e; }",
                               "if (prev[e] < best) { best = prev[e]; best_e = e; }"),
    "filter_free_read_start": ("cur[0] = (int64_t)r;", "cur[0] = 0;"),
    "filter_strings_not_reversed": ("const uint8_t tc = T[n - e];", "const uint8_t tc = T[e - 1];"),
}

PIN_TESTS = [
    (pins.test_hand_examples, ("improved",)),
    (pins.test_hand_examples, ("uncompressed",)),
    (pins.test_sellers_matches_breadth_first_search, ()),
    (pins.test_dc_bits_mean_prefix_anchored_distance, ()),
    (pins.test_single_window_equals_sellers, ()),
    (pins.test_improved_equals_uncompressed_fuzz, ()),
    (pins.test_check_cigar_rejects_wrong_alignments, ()),
    (pins.test_filter_matches_brute_force, ()),
]


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name):
    old, new = MUTANTS[name]
    src = open(oracle.SRC).read()
    assert src.count(old) == 1, f"mutation site for {name} not found exactly once"
    with tempfile.TemporaryDirectory() as tmp:
        path = os.path.join(tmp, "genasm_oracle.c")
        with open(path, "w") as f:
            f.write(src.replace(old, new))
        so = oracle.compile_source(path, os.path.join(tmp, "libmutant.so"))
        saved = oracle._lib
        oracle._lib = oracle.load(so)
        caught = []
        try:
            for fn, args in PIN_TESTS:
                try:
                    fn(oracle, *args)
                except Exception as e:  # noqa: BLE001 - any failure counts as caught
                    caught.append((fn.__name__, type(e).__name__))
        finally:
            oracle._lib = saved
    assert caught, f"mutant {name} passed every pin"
