/*
 * CPU oracle for windowed GenASM alignment (DC + TB) and its improved form.
 *
 * TEST INFRASTRUCTURE ONLY: see genasm_oracle.h. Plain, slow, scalar C; no
 * blocking, fusion or reordering beyond what the algorithm states.
 *
 * What is computed. The paper (Introduction) improves GenASM, the Bitap-based
 * aligner it cites (Senol Cali et al., MICRO 2020): a DP table of
 * bitvectors R[d] is built (GenASM-DC) and a traceback walks it to recover the
 * alignment (GenASM-TB). The paper gives three improvements:
 *   (1) store, per DP entry, only the bitwise AND of its match, substitution,
 *       insertion and deletion bitvectors (the entry's R word) instead of the
 *       four vectors;
 *   (2) stop computing rows once an earlier row already holds the full
 *       solution (early exit);
 *   (3) do not store entries that traceback cannot reach.
 * The DC/TB definitions themselves are not in the paper; this file follows
 * the Bitap (Wu-Manber) edit-distance recurrence in GenASM's form:
 *   - bit p of a word stands for pattern-window character Pw[mw-1-p] (so the
 *     most significant used bit is the first pattern character), 0 = match;
 *   - the text window is scanned from its last character to its first, so the
 *     traceback walks forward from text position 0;
 *   - R[d][i] bit p == 0 iff the pattern suffix Pw[mw-1-p .. mw) aligns to a
 *     prefix of Tw[i ..] with at most d unit-cost edits.
 *   - column n (past the text end) holds ~0 << d: only the pattern characters
 *     that d insertions can absorb match there.
 *   - row 0:      R[0][i] = (R[0][i+1] << 1) | PM[T[i]]
 *     row d >= 1: match        = (R[d][i+1]   << 1) | PM[T[i]]
 *                 substitution =  R[d-1][i+1] << 1
 *                 insertion    =  R[d-1][i]   << 1   (read base with no reference base)
 *                 deletion     =  R[d-1][i+1]        (reference base with no read base)
 *                 R[d][i] = match & substitution & insertion & deletion
 * Windowing: a read is aligned in windows of at most W pattern and W text
 * characters; the traceback of each window commits at most W-O characters of
 * either sequence, and the next window starts where it stopped.
 */
#define _POSIX_C_SOURCE 200809L
#include "genasm_oracle.h"

#include <pthread.h>
#include <stdatomic.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>
#include <unistd.h>

/* Column past the text end of row d: ~0 << d, and 0 for d >= 64 (a shift by
 * 64 or more is undefined in C). */
static uint64_t init_word(int d) { return d >= 64 ? 0 : (~0ull << d); }

static int bit_is_zero(uint64_t w, int p) { return ((w >> p) & 1ull) == 0; }

/* Pattern masks: bit q of pm[c] is 0 iff Pw[mw-1-q] == c. Bits >= mw stay 1;
 * left shifts never move them into the used range. */
static void build_pm(const uint8_t* Pw, int mw, uint64_t pm[4]) {
    for (int c = 0; c < 4; ++c) pm[c] = ~0ull;
    for (int q = 0; q < mw; ++q) pm[Pw[mw - 1 - q]] &= ~(1ull << q);
}

/* One DC cell, written as the AND of its four edge bitvectors. */
static uint64_t dc_cell(int d, uint64_t r_same_right, uint64_t r_up_right, uint64_t r_up_here,
                        uint64_t pm_t) {
    uint64_t match = (r_same_right << 1) | pm_t;
    if (d == 0) return match;
    uint64_t substitution = r_up_right << 1;
    uint64_t insertion = r_up_here << 1;
    uint64_t deletion = r_up_right;
    return match & substitution & insertion & deletion;
}

/* ------------------------------------------------------------------------ */
/* Infix (Sellers) edit distance.                                            */
/* ------------------------------------------------------------------------ */
int64_t oracle_sellers(const uint8_t* P, uint32_t m, const uint8_t* T, uint32_t n) {
    int64_t* prev = malloc(sizeof(int64_t) * ((size_t)n + 1));
    int64_t* cur = malloc(sizeof(int64_t) * ((size_t)n + 1));
    if (!prev || !cur) { free(prev); free(cur); return -1; }
    /* C[r][j] = min over a of Lev(P[0..r), T[a..j)); a free start is C[0][j] = 0. */
    for (uint32_t j = 0; j <= n; ++j) prev[j] = 0;
    for (uint32_t r = 1; r <= m; ++r) {
        cur[0] = r;
        for (uint32_t j = 1; j <= n; ++j) {
            int64_t diag = prev[j - 1] + (P[r - 1] != T[j - 1]);
            int64_t up = prev[j] + 1;
            int64_t left = cur[j - 1] + 1;
            int64_t best = diag < up ? diag : up;
            cur[j] = best < left ? best : left;
        }
        int64_t* t = prev; prev = cur; cur = t;
    }
    int64_t best = prev[0];
    for (uint32_t j = 1; j <= n; ++j) if (prev[j] < best) best = prev[j];
    free(prev); free(cur);
    return best;
}

int32_t oracle_filter(const uint8_t* P, uint32_t m, const uint8_t* T, uint32_t n, int32_t k,
                      uint32_t* start) {
    /* Reversed read P' and reference T': Lev(P, T[a..b)) = Lev(P', T'[n-b..n-a)).
     * C[r][e] = min over s of Lev(P'[0..r), T'[s..e)), free start C[0][e] = 0;
     * then the best substring starting at a costs C[m][n-a]. */
    int64_t* prev = malloc(sizeof(int64_t) * ((size_t)n + 1));
    int64_t* cur = malloc(sizeof(int64_t) * ((size_t)n + 1));
    if (!prev || !cur) { free(prev); free(cur); return -2; }
    for (uint32_t e = 0; e <= n; ++e) prev[e] = 0;
    for (uint32_t r = 1; r <= m; ++r) {
        const uint8_t pc = P[m - r];  /* P'[r-1] */
        cur[0] = (int64_t)r;          /* r read bases against an empty substring */
        for (uint32_t e = 1; e <= n; ++e) {
            const uint8_t tc = T[n - e];  /* T'[e-1] */
            int64_t diag = prev[e - 1] + (pc != tc);
            int64_t up = prev[e] + 1;
            int64_t left = cur[e - 1] + 1;
            int64_t best = diag < up ? diag : up;
            cur[e] = best < left ? best : left;
        }
        int64_t* t = prev; prev = cur; cur = t;
    }
    int64_t best = prev[0];
    uint32_t best_e = 0;
    for (uint32_t e = 1; e <= n; ++e) {
        if (prev[e] <= best) { best = prev[e]; best_e = e; }  /* largest e: least a */
    }
    free(prev); free(cur);
    if (best > k) return -1;
    if (start) *start = n - best_e;
    return (int32_t)best;
}

/* ------------------------------------------------------------------------ */
/* CIGAR replay.                                                             */
/* ------------------------------------------------------------------------ */
int oracle_check_cigar(const uint8_t* P, uint32_t m, const uint8_t* T, uint32_t n,
                       uint32_t begin, uint32_t end, const char* ops, uint32_t n_ops,
                       int32_t score) {
    if (begin > end || end > n) return -1;
    uint64_t pi = 0, ti = begin;
    int64_t edits = 0;
    for (uint32_t k = 0; k < n_ops; ++k) {
        switch (ops[k]) {
            case '=':
                if (pi >= m || ti >= end) return -2;
                if (P[pi] != T[ti]) return -3;
                ++pi; ++ti; break;
            case 'X':
                if (pi >= m || ti >= end) return -2;
                if (P[pi] == T[ti]) return -4;
                ++pi; ++ti; ++edits; break;
            case 'I':
                if (pi >= m) return -2;
                ++pi; ++edits; break;
            case 'D':
                if (ti >= end) return -2;
                ++ti; ++edits; break;
            default: return -5;
        }
    }
    if (pi != m) return -6;
    if (ti != end) return -7;
    if (edits != score) return -8;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Start-location search: DC only, first pattern window against the whole    */
/* reference. Returns the least row d <= K in which some column i in [0, n]  */
/* has a zero most significant bit, and the least such column in *col.       */
/* ------------------------------------------------------------------------ */

/* Improved form: row by row, stopping at the first row with a hit. */
static int search_improved(const uint8_t* P, int m1, const uint8_t* T, uint32_t n, int K,
                           uint32_t* col, oracle_result* res) {
    uint64_t pm[4];
    build_pm(P, m1, pm);
    const uint64_t msb = 1ull << (m1 - 1);
    uint64_t* prev = malloc(sizeof(uint64_t) * ((size_t)n + 1));
    uint64_t* cur = malloc(sizeof(uint64_t) * ((size_t)n + 1));
    if (!prev || !cur) { free(prev); free(cur); return -2; }
    int found = -1;
    for (int d = 0; d <= K && found < 0; ++d) {
        cur[n] = init_word(d);
        for (int64_t i = (int64_t)n - 1; i >= 0; --i)
            cur[i] = dc_cell(d, cur[i + 1], d ? prev[i + 1] : 0, d ? prev[i] : 0, pm[T[i]]);
        for (uint32_t i = 0; i <= n; ++i) {
            if (!(cur[i] & msb)) { found = d; *col = i; break; }
        }
        uint64_t* t = prev; prev = cur; cur = t;
    }
    free(prev); free(cur);
    return found;
}

/* Uncompressed form: column by column over all rows 0..K, then the least row. */
static int search_uncompressed(const uint8_t* P, int m1, const uint8_t* T, uint32_t n, int K,
                               uint32_t* col, oracle_result* res) {
    (void)res;
    uint64_t pm[4];
    build_pm(P, m1, pm);
    const uint64_t msb = 1ull << (m1 - 1);
    uint64_t* right = malloc(sizeof(uint64_t) * (K + 1));
    uint64_t* here = malloc(sizeof(uint64_t) * (K + 1));
    int64_t* leftmost = malloc(sizeof(int64_t) * (K + 1));
    if (!right || !here || !leftmost) { free(right); free(here); free(leftmost); return -2; }
    for (int d = 0; d <= K; ++d) {
        right[d] = init_word(d);
        leftmost[d] = (right[d] & msb) ? -1 : (int64_t)n;
    }
    for (int64_t i = (int64_t)n - 1; i >= 0; --i) {
        for (int d = 0; d <= K; ++d) {
            here[d] = dc_cell(d, right[d], d ? right[d - 1] : 0, d ? here[d - 1] : 0, pm[T[i]]);
            if (!(here[d] & msb)) leftmost[d] = i;
        }
        uint64_t* t = right; right = here; here = t;
    }
    int found = -1;
    for (int d = 0; d <= K; ++d) {
        if (leftmost[d] >= 0) { found = d; *col = (uint32_t)leftmost[d]; break; }
    }
    free(right); free(here); free(leftmost);
    return found;
}

/* ------------------------------------------------------------------------ */
/* One window: DC then TB.                                                   */
/* ------------------------------------------------------------------------ */

typedef struct {
    int i_end;      /* text characters consumed */
    int j_end;      /* pattern characters consumed */
    int edits;      /* edits committed */
    int n_ops;
    int status;
} window_out;

/* Traceback state machine shared in shape by both forms: from (i=0, p=mw-1,
 * d=dstar), take the first valid edge in the order match, substitution,
 * insertion, deletion, until the pattern window is consumed or W-O
 * characters of either sequence have been committed. The edge tests are
 * supplied by the form through `edge_ok`. */
typedef int (*edge_fn)(void* ctx, int edge, int d, int i, int p, int* status);

enum { EDGE_M = 0, EDGE_S = 1, EDGE_I = 2, EDGE_D = 3 };

static window_out traceback(void* ctx, edge_fn edge_ok, const uint8_t* Pw, int mw,
                            const uint8_t* Tw, int nw, int dstar, int L, char* ops, int ops_cap) {
    window_out w = {0, 0, 0, 0, 0};
    int i = 0, p = mw - 1, d = dstar, j = 0;
    while (p >= 0 && i < L && j < L) {
        char op;
        int st = 0;
        if (i < nw && Pw[j] == Tw[i] && edge_ok(ctx, EDGE_M, d, i, p, &st)) {
            op = '='; ++i; --p;
        } else if (st == 0 && d >= 1 && i < nw && edge_ok(ctx, EDGE_S, d, i, p, &st)) {
            op = 'X'; ++i; --p; --d;
        } else if (st == 0 && d >= 1 && edge_ok(ctx, EDGE_I, d, i, p, &st)) {
            op = 'I'; --p; --d;
        } else if (st == 0 && d >= 1 && i < nw && edge_ok(ctx, EDGE_D, d, i, p, &st)) {
            op = 'D'; ++i; --d;
        } else {
            w.status = st ? st : -2;
            return w;
        }
        if (st) { w.status = st; return w; }
        if (w.n_ops >= ops_cap) { w.status = -4; return w; }
        ops[w.n_ops++] = op;
        j = mw - 1 - p;
    }
    w.i_end = i;
    w.j_end = j;
    w.edits = dstar - d;
    return w;
}

/* Improved form: the table holds only R (improvement 1), rows 0..d* (2),
 * columns 0..min(nw, W-O) (3). */
typedef struct {
    const uint64_t* table;  /* rows 0..rows-1, each `cols` words */
    int rows, cols;
    int nw;
    oracle_result* res;
} improved_tb;

static int improved_read(improved_tb* c, int d, int i, uint64_t* out) {
    if (d < 0 || d >= c->rows || i < 0 || i >= c->cols) return -3;
    c->res->words_read++;
    *out = c->table[(size_t)d * c->cols + i];
    return 0;
}

/* The edge words are recomputed from the stored R words: bit p of
 *   match        is 0 iff the bases are equal and (p == 0 or bit p-1 of R[d][i+1] is 0),
 *   substitution is 0 iff p == 0 or bit p-1 of R[d-1][i+1] is 0,
 *   insertion    is 0 iff p == 0 or bit p-1 of R[d-1][i] is 0,
 *   deletion     is 0 iff bit p of R[d-1][i+1] is 0.
 * (The base comparison of the match edge is made by the caller.) */
static int improved_edge(void* vctx, int edge, int d, int i, int p, int* status) {
    improved_tb* c = vctx;
    uint64_t w;
    switch (edge) {
        case EDGE_M:
            if (p == 0) return 1;
            if ((*status = improved_read(c, d, i + 1, &w))) return 0;
            return bit_is_zero(w, p - 1);
        case EDGE_S:
            if (p == 0) return 1;
            if ((*status = improved_read(c, d - 1, i + 1, &w))) return 0;
            return bit_is_zero(w, p - 1);
        case EDGE_I:
            if (p == 0) return 1;
            if ((*status = improved_read(c, d - 1, i, &w))) return 0;
            return bit_is_zero(w, p - 1);
        default:
            if ((*status = improved_read(c, d - 1, i + 1, &w))) return 0;
            return bit_is_zero(w, p);
    }
}

static window_out window_improved(const uint8_t* Pw, int mw, const uint8_t* Tw, int nw, int K,
                                  int L, char* ops, int ops_cap, oracle_result* res) {
    window_out w = {0, 0, 0, 0, 0};
    uint64_t pm[4];
    build_pm(Pw, mw, pm);
    const uint64_t msb = 1ull << (mw - 1);
    const int cols = (nw < L ? nw : L) + 1;  /* stored columns 0..min(nw, L) */
    uint64_t* prev = malloc(sizeof(uint64_t) * (nw + 1));
    uint64_t* cur = malloc(sizeof(uint64_t) * (nw + 1));
    uint64_t* table = malloc(sizeof(uint64_t) * (size_t)(K + 1) * cols);
    if (!prev || !cur || !table) {
        free(prev); free(cur); free(table);
        w.status = -5;
        return w;
    }
    int dstar = -1;
    for (int d = 0; d <= K; ++d) {
        cur[nw] = init_word(d);
        for (int i = nw - 1; i >= 0; --i)
            cur[i] = dc_cell(d, cur[i + 1], d ? prev[i + 1] : 0, d ? prev[i] : 0, pm[Tw[i]]);
        res->rows_window++;
        res->word_ops += (uint64_t)nw * (d ? 6 : 2);
        memcpy(table + (size_t)d * cols, cur, sizeof(uint64_t) * cols);
        res->words_stored += cols;
        if (!(cur[0] & msb)) { dstar = d; break; }  /* early exit */
        uint64_t* t = prev; prev = cur; cur = t;
    }
    if (dstar < 0) {
        w.status = 1;  /* no solution within K */
    } else {
        uint64_t words = (uint64_t)(dstar + 1) * cols;
        if (words > res->words_peak) res->words_peak = words;
        improved_tb ctx = {table, dstar + 1, cols, nw, res};
        w = traceback(&ctx, improved_edge, Pw, mw, Tw, nw, dstar, L, ops, ops_cap);
    }
    free(prev); free(cur); free(table);
    return w;
}

/* Uncompressed form: every entry (d, i), d in 0..K, i in 0..nw-1, keeps its
 * four edge words; d* is read off afterwards; traceback tests edge bits. */
typedef struct {
    const uint64_t* edges;  /* [(d * nw + i) * 4 + edge] */
    int K, nw;
    oracle_result* res;
} uncompressed_tb;

static int uncompressed_edge(void* vctx, int edge, int d, int i, int p, int* status) {
    uncompressed_tb* c = vctx;
    uint64_t w;
    if (i == c->nw) {
        /* Past the text end only the insertion edge exists; it derives from
         * the column's initial value ~0 << (d-1). */
        if (edge != EDGE_I) { *status = -3; return 0; }
        w = init_word(d - 1) << 1;
        return bit_is_zero(w, p);
    }
    if (d < 0 || d > c->K || i < 0 || i >= c->nw) { *status = -3; return 0; }
    c->res->words_read++;
    w = c->edges[((size_t)d * c->nw + i) * 4 + edge];
    return bit_is_zero(w, p);
}

static window_out window_uncompressed(const uint8_t* Pw, int mw, const uint8_t* Tw, int nw, int K,
                                      int L, char* ops, int ops_cap, oracle_result* res) {
    window_out w = {0, 0, 0, 0, 0};
    uint64_t pm[4];
    build_pm(Pw, mw, pm);
    const uint64_t msb = 1ull << (mw - 1);
    uint64_t* right = malloc(sizeof(uint64_t) * (K + 1));
    uint64_t* here = malloc(sizeof(uint64_t) * (K + 1));
    uint64_t* edges = malloc(sizeof(uint64_t) * 4 * (size_t)(K + 1) * (nw > 0 ? nw : 1));
    if (!right || !here || !edges) {
        free(right); free(here); free(edges);
        w.status = -5;
        return w;
    }
    for (int d = 0; d <= K; ++d) right[d] = init_word(d);
    for (int i = nw - 1; i >= 0; --i) {
        for (int d = 0; d <= K; ++d) {
            uint64_t* e = edges + ((size_t)d * nw + i) * 4;
            e[EDGE_M] = (right[d] << 1) | pm[Tw[i]];
            res->words_stored++;
            if (d == 0) {
                here[d] = e[EDGE_M];
                res->word_ops += 2;
                continue;
            }
            e[EDGE_S] = right[d - 1] << 1;
            e[EDGE_I] = here[d - 1] << 1;
            e[EDGE_D] = right[d - 1];
            res->words_stored += 3;
            here[d] = e[EDGE_M] & e[EDGE_S] & e[EDGE_I] & e[EDGE_D];
            res->word_ops += 6;
        }
        uint64_t* t = right; right = here; here = t;
    }
    res->rows_window += K + 1;
    /* After the loop, right[] holds column 0 (or the initial column if nw == 0). */
    int dstar = -1;
    for (int d = 0; d <= K; ++d) {
        if (!(right[d] & msb)) { dstar = d; break; }
    }
    uint64_t words = (uint64_t)4 * (K + 1) * nw;
    if (words > res->words_peak) res->words_peak = words;
    if (dstar < 0) {
        w.status = 1;
    } else {
        uncompressed_tb ctx = {edges, K, nw, res};
        w = traceback(&ctx, uncompressed_edge, Pw, mw, Tw, nw, dstar, L, ops, ops_cap);
    }
    free(right); free(here); free(edges);
    return w;
}

/* ------------------------------------------------------------------------ */
/* Whole-read alignment.                                                     */
/* ------------------------------------------------------------------------ */
int oracle_align(int variant, const uint8_t* P, uint32_t m, const uint8_t* T, uint32_t n,
                 int32_t k, int32_t W, int32_t O, char* ops, uint32_t ops_cap,
                 oracle_result* res) {
    memset(res, 0, sizeof(*res));
    res->d_min = -1;
    if (W < 2 || W > 64 || O < 0 || O >= W || k < 0) { res->status = -1; res->score = -1; return -1; }
    if (m == 0) return 0;
    const int K = k < W ? k : W;
    const int L = W - O;

    /* Start location: least edit row, then leftmost column. */
    const int m1 = (int)(m < (uint32_t)W ? m : (uint32_t)W);
    uint32_t s = 0;
    int dmin = variant == ORACLE_IMPROVED ? search_improved(P, m1, T, n, K, &s, res)
                                          : search_uncompressed(P, m1, T, n, K, &s, res);
    res->cells_search = (uint64_t)m1 * n;
    if (dmin == -2) { res->status = -5; res->score = -1; return -5; }
    res->d_min = dmin;
    res->search_col = s;
    if (dmin < 0) { res->score = -1; return 0; }

    uint64_t ti = s, pj = 0;
    int64_t score = 0;
    uint32_t n_ops = 0;
    while (pj < m) {
        const int mw = (int)((m - pj) < (uint64_t)W ? (m - pj) : (uint64_t)W);
        const int nw = (int)((n - ti) < (uint64_t)W ? (n - ti) : (uint64_t)W);
        res->n_windows++;
        res->cells_window += (uint64_t)mw * nw;
        window_out w = variant == ORACLE_IMPROVED
            ? window_improved(P + pj, mw, T + ti, nw, K, L, ops + n_ops, (int)(ops_cap - n_ops), res)
            : window_uncompressed(P + pj, mw, T + ti, nw, K, L, ops + n_ops, (int)(ops_cap - n_ops), res);
        if (w.status == 1) {  /* window without a solution within K: the pair fails */
            res->score = -1;
            res->n_ops = 0;
            res->ref_begin = res->ref_end = 0;
            return 0;
        }
        if (w.status) { res->status = w.status; res->score = -1; return w.status; }
        score += w.edits;
        n_ops += w.n_ops;
        ti += w.i_end;
        pj += w.j_end;
    }
    res->score = (int32_t)score;
    res->n_ops = n_ops;
    res->ref_begin = s;
    res->ref_end = (uint32_t)ti;
    return 0;
}

int oracle_dc_rows(const uint8_t* P, uint32_t m1, const uint8_t* T, uint32_t n, int32_t K,
                   uint64_t* out) {
    if (m1 < 1 || m1 > 64 || K < 0) return -1;
    uint64_t pm[4];
    build_pm(P, (int)m1, pm);
    const size_t cols = (size_t)n + 1;
    for (int d = 0; d <= K; ++d) {
        uint64_t* cur = out + (size_t)d * cols;
        const uint64_t* prev = d ? out + (size_t)(d - 1) * cols : NULL;
        cur[n] = init_word(d);
        for (int64_t i = (int64_t)n - 1; i >= 0; --i)
            cur[i] = dc_cell(d, cur[i + 1], d ? prev[i + 1] : 0, d ? prev[i] : 0, pm[T[i]]);
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Threaded batch driver (timing baseline).                                  */
/* ------------------------------------------------------------------------ */
typedef struct {
    int variant;
    const uint8_t *reads, *refs;
    const uint64_t *read_off, *ref_off;
    uint64_t n_pairs;
    int32_t k, W, O;
    char* ops;
    oracle_result* res;
    atomic_uint_fast64_t next;
} batch_job;

static void* batch_worker(void* arg) {
    batch_job* j = arg;
    for (;;) {
        uint64_t i = atomic_fetch_add(&j->next, 1);
        if (i >= j->n_pairs) break;
        uint64_t m = j->read_off[i + 1] - j->read_off[i];
        uint64_t n = j->ref_off[i + 1] - j->ref_off[i];
        oracle_align(j->variant, j->reads + j->read_off[i], (uint32_t)m, j->refs + j->ref_off[i],
                     (uint32_t)n, j->k, j->W, j->O, j->ops + j->read_off[i] + j->ref_off[i],
                     (uint32_t)(m + n), &j->res[i]);
    }
    return NULL;
}

double oracle_batch(int variant, const uint8_t* reads, const uint64_t* read_off,
                    const uint8_t* refs, const uint64_t* ref_off, uint64_t n_pairs,
                    int32_t k, int32_t W, int32_t O, int nthreads, char* ops,
                    oracle_result* res, int* threads_used) {
    if (nthreads <= 0) nthreads = (int)sysconf(_SC_NPROCESSORS_ONLN);
    if (nthreads < 1) nthreads = 1;
    batch_job job;
    job.variant = variant;
    job.reads = reads;
    job.refs = refs;
    job.read_off = read_off;
    job.ref_off = ref_off;
    job.n_pairs = n_pairs;
    job.k = k;
    job.W = W;
    job.O = O;
    job.ops = ops;
    job.res = res;
    atomic_init(&job.next, 0);
    pthread_t* th = malloc(sizeof(pthread_t) * nthreads);
    struct timespec t0, t1;
    clock_gettime(CLOCK_MONOTONIC, &t0);
    int started = 0;
    for (int t = 0; t < nthreads; ++t)
        if (pthread_create(&th[t], NULL, batch_worker, &job) == 0) ++started;
    if (started == 0) batch_worker(&job);
    for (int t = 0; t < started; ++t) pthread_join(th[t], NULL);
    clock_gettime(CLOCK_MONOTONIC, &t1);
    free(th);
    if (threads_used) *threads_used = started ? started : 1;
    return (double)(t1.tv_sec - t0.tv_sec) + 1e-9 * (double)(t1.tv_nsec - t0.tv_nsec);
}
