/*
 * CPU oracle for windowed GenASM alignment (DC + TB).
 *
 * TEST INFRASTRUCTURE ONLY. This library exists to check the GPU library's
 * outputs. Only the test suite, the smoke check and the benchmark's CPU
 * baseline leg may load it; the product path never calls it, and it shares
 * no code, header or table with the GPU library.
 *
 * Sequences are arrays of base codes A=0, C=1, G=2, T=3.
 *
 * Parity status of each function (pins live in tests/test_oracle_*.py):
 *   oracle_sellers        pinned: brute-force breadth-first edit search on
 *                         tiny inputs, exact-occurrence and empty-text
 *                         closed forms.
 *   oracle_align          pinned on single-window inputs to oracle_sellers
 *                         (windowing is exact there), by CIGAR replay, by
 *                         the Sellers lower bound, by row invariants and by
 *                         hand-worked examples. Multi-window CIGAR choice is
 *                         "parity unpinned": no external source fixes it
 *                         beyond those properties.
 *   oracle_check_cigar    pinned by planted mistakes in tests.
 *   oracle_filter         pinned: brute-force minimum over all substrings
 *                         (distance and leftmost start) on tiny inputs,
 *                         exact-occurrence and empty-read closed forms, and
 *                         equality with oracle_sellers.
 */
#ifndef GENASM_ORACLE_H
#define GENASM_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    ORACLE_IMPROVED = 0,     /* store only the AND, early exit, pruned table */
    ORACLE_UNCOMPRESSED = 1  /* four edge words per entry, all rows, all columns */
};

typedef struct {
    int32_t score;         /* edit distance, -1 when some window has no solution within k */
    uint32_t ref_begin;    /* reference span [ref_begin, ref_end) covered by the alignment */
    uint32_t ref_end;
    uint32_t n_windows;    /* windows processed */
    uint32_t n_ops;        /* ops written ('=', 'X', 'I', 'D') */
    int32_t status;        /* 0 = ok; -2 = traceback found no valid edge; -3 = traceback read
                              outside the stored table; -4 = ops buffer too small; -5 = no memory */
    int32_t d_min;         /* start search: least row with a hit (-1 if none) */
    uint32_t search_col;   /* start search: leftmost hit column */
    /* Table instrumentation, summed over windows. */
    uint64_t words_stored;     /* DP-table words written */
    uint64_t words_read;       /* DP-table words read by traceback */
    uint64_t words_peak;       /* largest single-window table, in words */
    uint64_t cells_window;     /* sum over windows of m_w * n_w */
    uint64_t cells_search;     /* m1 * n */
    uint64_t rows_window;      /* DC rows computed, summed over windows */
    uint64_t word_ops;         /* 64-bit DC word operations (2 per row-0 cell, 6 per other cell) */
} oracle_result;

/* Align read P[0..m) to reference T[0..n) with error cap k, window W,
 * overlap O. Writes ops into ops[0..ops_cap). Returns res->status. */
int oracle_align(int variant, const uint8_t* P, uint32_t m, const uint8_t* T, uint32_t n,
                 int32_t k, int32_t W, int32_t O, char* ops, uint32_t ops_cap,
                 oracle_result* res);

/* Infix (Sellers) edit distance: min over a <= b of Levenshtein(P, T[a..b)). */
/* Pre-alignment filter (score-only mode): d = the least edit distance between
 * the whole read P and any substring T[a..b) of the reference. Returns d when
 * d <= k, else -1; *start receives the least a with min_b Lev(P, T[a..b)) = d
 * (when d <= k). Definition written out: a Sellers DP over the reversed
 * strings, whose free start becomes the free end of the substring. */
int32_t oracle_filter(const uint8_t* P, uint32_t m, const uint8_t* T, uint32_t n, int32_t k,
                      uint32_t* start);

int64_t oracle_sellers(const uint8_t* P, uint32_t m, const uint8_t* T, uint32_t n);

/* Replays ops against P and T[begin..end). Returns 0 when the ops turn P into
 * T[begin..end) with '=' only on equal bases, 'X' only on unequal ones and
 * exactly `score` edits; a negative code naming the first violation otherwise. */
int oracle_check_cigar(const uint8_t* P, uint32_t m, const uint8_t* T, uint32_t n,
                       uint32_t begin, uint32_t end, const char* ops, uint32_t n_ops,
                       int32_t score);

/* Aligns pairs [0, n_pairs) on `nthreads` threads (0 = all cores). Pair i's ops
 * go to ops + read_off[i] + ref_off[i] (room for m + n ops). Returns the wall
 * time of the alignment loop in seconds; *threads_used receives the count. */
double oracle_batch(int variant, const uint8_t* reads, const uint64_t* read_off,
                    const uint8_t* refs, const uint64_t* ref_off, uint64_t n_pairs,
                    int32_t k, int32_t W, int32_t O, int nthreads, char* ops,
                    oracle_result* res, int* threads_used);

/* Row invariants of the DC recurrence, for tests: computes rows 0..K of one
 * window over the whole text (no early exit) into out[(K+1)*(n+1)] and
 * returns 0. Row d, column i is out[d*(n+1)+i]. */
int oracle_dc_rows(const uint8_t* P, uint32_t m1, const uint8_t* T, uint32_t n, int32_t K,
                   uint64_t* out);

#ifdef __cplusplus
}
#endif

#endif
