/*
 * genasm.h - C ABI of the gfx950 GenASM aligner (windowed bit-parallel
 * edit-distance calculation, GenASM-DC, plus traceback, GenASM-TB, with the
 * three improvements of Lindegger et al., "Algorithmic Improvement and GPU
 * Acceleration of the GenASM Algorithm", 2022).
 *
 * The operation (paper, Introduction): build the DP table of bitvectors R[d]
 * for each window of a (read, reference) pair, then trace back through it to
 * recover the alignment, storing per DP entry only the AND of its four edge
 * bitvectors (key idea 1), stopping once a row holds the full solution (key
 * idea 2) and never storing entries the traceback cannot reach (key idea 3).
 * The paper's Results section aligns (read, reference) candidate pairs; this
 * library aligns batches of such pairs, one result and one CIGAR per pair.
 *
 * Semantics, in the notation of the GenASM recurrence (0 = match, bit p of a
 * word stands for pattern character Pw[mw-1-p]):
 *   - K = min(k, W) caps the rows of every window and of the start search.
 *   - The alignment starts at the least edit row, then the leftmost column,
 *     in which the first read window (at most W bases) fits anywhere in the
 *     reference (start search).
 *   - Windows of at most W read and W reference bases follow; each window's
 *     traceback takes the first valid edge in the order match, substitution,
 *     insertion, deletion, and commits at most W-O bases of either sequence.
 *   - A window with no solution within K fails the pair: edit_distance = -1,
 *     empty CIGAR, ref_begin = ref_end = 0.
 *   - A read of length 0 gives edit_distance 0, an empty CIGAR, span [0,0).
 * CIGAR ops are '=', 'X', 'I' (read base absent from the reference) and 'D'
 * (reference base absent from the read); runs merge across window seams.
 *
 * Testing the error paths: with the environment variable GENASM_FAIL_ALLOC
 * set to 1, every device allocation the library would make (a context buffer
 * that has to grow, a server's pools) fails as if the device were full, so
 * the calls return GENASM_E_NOMEM and leave the context usable.
 *
 * Threading: a genasm_ctx is not thread-safe; use one per host thread.
 * No C++ exception crosses this interface. Every call returns GENASM_OK (0)
 * or a negative error code.
 */
#ifndef GENASM_H
#define GENASM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GENASM_ABI_VERSION 1

/* Error codes. */
#define GENASM_OK 0
#define GENASM_E_INVAL (-1)     /* bad argument: W not in [2,64], O not in [0,W-1], k < 0,
                                   null pointer, offsets not non-decreasing, bad launch */
#define GENASM_E_ALPHABET (-2)  /* a sequence byte outside A,C,G,T,a,c,g,t */
#define GENASM_E_NOMEM (-3)     /* host or device allocation failed */
#define GENASM_E_DEVICE (-4)    /* HIP error; genasm_last_error() has the message */
#define GENASM_E_NOSPACE (-5)   /* output buffer too small; the needed size is reported */
#define GENASM_E_BUSY (-6)      /* serving: request refused, admission budget exhausted */
#define GENASM_E_TOOLONG (-7)   /* a sequence is longer than 2^31 - 1 bases */
#define GENASM_E_PINNED (-8)    /* the context's device buffers are held by a captured graph
                                   and the call would have to grow them (see genasm_unpin) */
#define GENASM_E_SCRATCH (-9)   /* genasm_batch_align_dev_noalloc: the batch needs more device
                                   scratch than GENASM_NOALLOC_SCRATCH_BYTES */

/* Per-pair result (the alignment the traceback retrieves: Introduction, the
 * traceback step; its edit count is the sum of the windows' committed edits).
 * 32 bytes, 8-byte aligned. */
typedef struct {
    int32_t edit_distance; /* total committed edits, -1 if some window had no solution within k */
    uint32_t ref_begin;    /* alignment covers reference bases [ref_begin, ref_end) */
    uint32_t ref_end;
    uint32_t n_windows;    /* windows processed (0 for an empty read or a failed start search) */
    uint64_t cigar_off;    /* first CIGAR element of this pair (see the two call forms) */
    uint32_t cigar_len;    /* CIGAR elements (device form) or characters (host form) */
    uint32_t flags;        /* GENASM_FLAG_* bits; 0 on success */
} genasm_result;

#define GENASM_FLAG_CIGAR_OVERFLOW 1u  /* device form: the CIGAR did not fit; cigar_len is 0 */
#define GENASM_FLAG_INTERNAL 2u        /* traceback found no valid edge, or (debug builds) a checked
                                          invariant failed for this pair; never expected */

/* Device-form CIGAR element: run length in bits 31..2, op in bits 1..0. */
#define GENASM_OP_MATCH 0u    /* '=' */
#define GENASM_OP_MISMATCH 1u /* 'X' */
#define GENASM_OP_INS 2u      /* 'I' */
#define GENASM_OP_DEL 3u      /* 'D' */
#define GENASM_CIGAR_LEN(e) ((e) >> 2)
#define GENASM_CIGAR_OP(e) ((e) & 3u)

/* Launch forms. */
#define GENASM_FORM_PLAIN 0    /* one pair per workgroup: 64 lanes = 64 DP rows of one pair */
#define GENASM_FORM_BATCHED 1  /* search kernels, then one persistent window kernel with a
                                  device work queue; several pairs per wavefront */
#define GENASM_FORM_UNIMPROVED 2 /* ablation: one pair per workgroup, each window computing
                                  every row 0..K and keeping the four edge words of every
                                  entry in device memory (no early exit, no AND, no pruning);
                                  same results, for measuring what the improvements save */

typedef struct {
    int32_t form;            /* GENASM_FORM_* */
    int32_t group_lanes;     /* batched: lanes (= DP rows per pass) per pair in the window
                                kernel for ordinary pairs, 16 or 64 (64 sends every pair to
                                the whole-wavefront path); 0 = default */
    int32_t search_lanes;    /* batched: lanes per pair in the start search, 16 or 64; 0 = default */
    int32_t lds_rows;        /* batched: window-table rows kept in LDS per 16-lane group
                                (16, 32, 48 or 64); rows above spill to device memory; 0 = default */
    int32_t workers_per_cu;  /* batched: resident window workgroups per compute unit; 0 = as many
                                as LDS allows */
    int32_t lpt_order;       /* batched: 1 = longest reads first, 0 = input order; -1 = default */
    int32_t hard_row;        /* batched: pairs whose start search needs this many edit rows or
                                more (decoy-like pairs, whose windows cost several DC passes)
                                go to a separate queue that the window workers drain first;
                                0 = default (16); -1 = every pair; 65 = no separate queue */
    int32_t hard_lanes;      /* batched: lanes per pair for that queue: 16 (the ordinary
                                groups, table rows past lds_rows spilled), 32 (two pairs per
                                wavefront, 32 rows per DC pass and in LDS; needs lds_rows
                                <= 48) or 64 (one pair per wavefront, the whole 64-row table
                                in LDS); 0 = default (16) */
    int32_t tb_prefetch;     /* batched: 1 = tracebacks over spilled rows load the next row
                                ahead through the group's lanes, 0 = one load per edit;
                                -1 = default */
    int32_t hard_share;      /* batched: percent (0..100) of the window workers that drain
                                the hard queue before the easy one (the others the other way
                                round); -1 = default (50) */
    int32_t table_bits;      /* batched, 16-lane groups for both queues: 32 = compact groups
                                (a window's table in LDS as 32-bit slices of its 16 rows,
                                valid while the window solves within 16 rows; a deeper
                                window is recomputed with 64-bit rows in device memory),
                                64 = 64-bit rows, lds_rows of them in LDS; 0 = default (64) */
    int32_t search_per_cu;   /* batched: start-search workgroups per compute unit (1..32);
                                0 = default (8) */
} genasm_launch;

typedef struct genasm_ctx genasm_ctx;

/* Creates a context on HIP device `hip_device`. The context owns a stream,
 * device scratch (grown on demand, reused across calls) and kernel handles.
 * Returns GENASM_E_DEVICE if no such device exists or it is not gfx950,
 * GENASM_E_NOMEM if the host allocation fails. (Library plumbing; the paper
 * defines no such object.) */
int genasm_create(genasm_ctx** out, int hip_device);

/* Frees everything the context owns. Safe on NULL. (Library plumbing.) */
void genasm_destroy(genasm_ctx* ctx);

/* Graph capture and the context's buffers (library plumbing around the device
 * form; no paper passage). A genasm_batch_align_dev call made
 * while its stream is being captured records kernels that use the context's
 * device buffers by address, so such a call pins the context: from then on a
 * call that would need larger buffers fails with GENASM_E_PINNED instead of
 * freeing them (size them first with an eager call of the largest shape).
 * genasm_unpin declares that no captured graph uses them any more (the graphs
 * were destroyed), after which calls may grow them again. Returns
 * GENASM_E_INVAL for a NULL context. */
int genasm_unpin(genasm_ctx* ctx);

/* Message of the last error on this context (never NULL). With ctx == NULL:
 * the reason of the calling thread's last failed genasm_create. (Library
 * plumbing.) */
const char* genasm_last_error(const genasm_ctx* ctx);

/* Static text for an error code. (Library plumbing.) */
const char* genasm_strerror(int code);

/* Fills *out with the default launch parameters of `form` (launch geometry of
 * the device form; library plumbing). Returns GENASM_E_INVAL for an unknown
 * form or a NULL out. */
int genasm_default_launch(int32_t form, genasm_launch* out);

/*
 * Host-memory form, synchronous. Defined by: the paper's Introduction (DP
 * table of GenASM-DC with key ideas 1-3, then GenASM-TB to retrieve the
 * alignment) applied to each (read, reference) candidate pair, as in its
 * Results section; windowing with W and O as in GenASM.
 *   reads, refs      ASCII sequences (ACGT, either case), concatenated.
 *   read_off,        n_pairs + 1 non-decreasing offsets: pair i is
 *   ref_off          reads[read_off[i] .. read_off[i+1]) against
 *                    refs[ref_off[i] .. ref_off[i+1]). read_off[0] may be
 *                    non-zero.
 *   k, W, O          error cap per window, window size (2..64), overlap (0..W-1).
 *   out              n_pairs results; cigar_off/cigar_len index cigar_buf.
 *   cigar_buf        CIGAR text of all pairs, back to back, no separators and no
 *                    terminating NUL (e.g. "12=1X3="); may be NULL when
 *                    cigar_cap == 0.
 *   cigar_needed     receives the number of characters the CIGARs need.
 *   launch           NULL for the default batched launch.
 * Returns GENASM_E_NOSPACE when cigar_cap < *cigar_needed: *cigar_needed is
 * set and nothing else is written (no partial results; call again with a
 * buffer of that size). GENASM_E_INVAL for bad k/W/O, null pointers or
 * decreasing offsets, GENASM_E_TOOLONG for a sequence of 2^31 bases or more,
 * GENASM_E_ALPHABET for a byte outside ACGTacgt, GENASM_E_NOMEM or
 * GENASM_E_DEVICE on allocation or HIP failure. The caller owns every buffer;
 * nothing is retained after the call returns.
 */
int genasm_batch_align(genasm_ctx* ctx, const char* reads, const uint64_t* read_off,
                       const char* refs, const uint64_t* ref_off, uint64_t n_pairs,
                       int32_t k, int32_t W, int32_t O, genasm_result* out, char* cigar_buf,
                       uint64_t cigar_cap, uint64_t* cigar_needed, const genasm_launch* launch);

/*
 * Device-memory form, asynchronous on `stream` (a hipStream_t; NULL = the
 * null stream). Defined by: as genasm_batch_align (Introduction, key ideas
 * 1-3 and the traceback step; Results, candidate pairs).
 *   d_reads2b,       2-bit packed sequences in device memory: base b of the
 *   d_refs2b         stream is bits 2*(b%4)..2*(b%4)+1 of byte b/4, codes
 *                    A=0, C=1, G=2, T=3 (see genasm_pack).
 *   d_read_off,      n_pairs + 1 non-decreasing base offsets, in device memory.
 *   d_ref_off
 *   d_out            n_pairs results in device memory.
 *   d_cigar          device CIGAR elements (GENASM_CIGAR_LEN/OP); pair i writes
 *                    at most m_i + n_i elements starting at element
 *                    (d_read_off[i] - d_read_off[0]) + (d_ref_off[i] - d_ref_off[0]),
 *                    where m_i, n_i are its read and reference lengths, so
 *                    cigar_cap must be at least (total read bases + total
 *                    reference bases); a pair whose CIGAR would pass cigar_cap
 *                    gets GENASM_FLAG_CIGAR_OVERFLOW.
 *   total_read_bases, total_ref_bases
 *                    d_read_off[n_pairs] - d_read_off[0] and the same for refs
 *                    (sizes the device scratch without a device-to-host copy).
 * The caller keeps every buffer alive until the stream has passed this call.
 * Scratch is owned by the context; calls on one context are serialized on
 * its device scratch, so do not run two calls of one context on different
 * streams at once. Errors (nothing is launched): GENASM_E_INVAL for bad
 * k/W/O, null pointers or launch parameters, GENASM_E_NOSPACE when cigar_cap
 * is below total_read_bases + total_ref_bases, GENASM_E_NOMEM when scratch
 * cannot grow, GENASM_E_PINNED when it would have to grow on a pinned context
 * (see genasm_unpin), GENASM_E_DEVICE on a HIP error. The call can be captured
 * into a HIP graph once the context's buffers are sized for its shape.
 */
int genasm_batch_align_dev(genasm_ctx* ctx, const uint8_t* d_reads2b, const uint64_t* d_read_off,
                           const uint8_t* d_refs2b, const uint64_t* d_ref_off, uint64_t n_pairs,
                           uint64_t total_read_bases, uint64_t total_ref_bases,
                           int32_t k, int32_t W, int32_t O,
                           genasm_result* d_out, uint32_t* d_cigar, uint64_t cigar_cap,
                           const genasm_launch* launch, void* stream);

/*
 * No-allocation variant of genasm_batch_align_dev, for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc. Arguments, layouts, ownership and results
 * are those of genasm_batch_align_dev, for the plain and batched forms. The
 * device scratch (bit planes of both streams, start-search items and keys,
 * window queues, the longest-first order, spilled window-table rows) comes
 * from a static device array of GENASM_NOALLOC_SCRATCH_BYTES that the library
 * holds on every device it runs on until the process ends; the call allocates
 * nothing (no hipMalloc, hipFree or allocating library routine) and does not
 * pin the context. With workers_per_cu = 0 the batched form runs the largest
 * resident window-worker count whose spill fits the array beside the batch.
 * The bit planes take about (total_read_bases + total_ref_bases) / 4 bytes;
 * the batched form adds about 40 bytes per pair and 0.3 bytes per reference
 * base, plus the spill of its window workers (16 KB each at W = 64, O = 24
 * with 16 table rows in LDS).
 * All calls on one device share the array, which keeps the last call's
 * contents; every call rewrites what it reads from it with kernels on its own
 * stream before reading. Calls that overlap in time on one device, from any
 * context or stream, race on it and give wrong results: serialize them.
 * Errors: as genasm_batch_align_dev, plus GENASM_E_SCRATCH (nothing is
 * launched; genasm_last_error gives the bytes needed) when the batch needs
 * more than the array, GENASM_E_INVAL for the unimproved form. Profiling
 * counters (genasm_profile_enable) are not recorded by this call.
 */
#define GENASM_NOALLOC_SCRATCH_BYTES (128ull << 20)
int genasm_batch_align_dev_noalloc(genasm_ctx* ctx, const uint8_t* d_reads2b,
                                   const uint64_t* d_read_off, const uint8_t* d_refs2b,
                                   const uint64_t* d_ref_off, uint64_t n_pairs,
                                   uint64_t total_read_bases, uint64_t total_ref_bases,
                                   int32_t k, int32_t W, int32_t O,
                                   genasm_result* d_out, uint32_t* d_cigar, uint64_t cigar_cap,
                                   const genasm_launch* launch, void* stream);

/*
 * Pre-alignment filter (score-only mode). Defined by: the Introduction's
 * place of edit-distance calculation ahead of alignment (pre-alignment
 * filtering), with GenASM-DC's recurrence: the DC recurrence over the whole
 * read, with no table and no traceback (GenASM-DC used as a filter ahead of
 * alignment, the use the paper's introduction gives for edit-distance
 * calculation). For pair i, dist[i] = the least edit distance between read i
 * and any substring of reference i when that is at most k, else -1; start[i]
 * = the least start of a reference substring at that distance (0 when
 * rejected). k is in [0, 63]; reads are at most 1024 bases (GENASM_E_TOOLONG
 * otherwise). Host form: ASCII streams and offsets as for genasm_batch_align,
 * synchronous. Device form: 2-bit packed streams and offsets in device memory
 * as for genasm_batch_align_dev, max_read_len an upper bound on the read
 * lengths, dist/start in device memory, asynchronous on `stream`.
 */
int genasm_filter(genasm_ctx* ctx, const char* reads, const uint64_t* read_off, const char* refs,
                  const uint64_t* ref_off, uint64_t n_pairs, int32_t k, int32_t* dist,
                  uint32_t* start);
int genasm_filter_dev(genasm_ctx* ctx, const uint8_t* d_reads2b, const uint64_t* d_read_off,
                      const uint8_t* d_refs2b, const uint64_t* d_ref_off, uint64_t n_pairs,
                      uint32_t max_read_len, int32_t k, int32_t* d_dist, uint32_t* d_start,
                      void* stream);

/*
 * Autotuner for the batched form (library plumbing, no paper passage: picks
 * the launch geometry of the device form). Runs the device-form call above on the given
 * batch with each candidate launch configuration (lanes per pair for the
 * decoy-like queue and its threshold row, the share of workers starting on
 * that queue, table rows kept in LDS, resident workers per compute unit, lanes
 * per pair in the start search, traceback prefetch), `reps` timed
 * runs each after one untimed run, and writes the fastest to *best (and its
 * time in ms to *best_ms if not NULL). Every run writes complete results, so
 * d_out/d_cigar hold the batch's alignment afterwards. The pick is cached in
 * the context under the batch's signature (pair count and mean read length to
 * the nearest power of two below, k, W, O); later genasm_batch_align_dev and
 * genasm_batch_align calls with launch == NULL and a matching signature use
 * it. Synchronizes `stream`.
 */
int genasm_autotune_dev(genasm_ctx* ctx, const uint8_t* d_reads2b, const uint64_t* d_read_off,
                        const uint8_t* d_refs2b, const uint64_t* d_ref_off, uint64_t n_pairs,
                        uint64_t total_read_bases, uint64_t total_ref_bases,
                        int32_t k, int32_t W, int32_t O, genasm_result* d_out, uint32_t* d_cigar,
                        uint64_t cigar_cap, int32_t reps, void* stream, genasm_launch* best,
                        float* best_ms);
/* Tuning cache as text, one signature per line; load merges into the context's
 * cache (library plumbing). GENASM_E_INVAL for a file that cannot be opened or
 * parsed; size returns the number of cached signatures. */
int genasm_tune_cache_save(genasm_ctx* ctx, const char* path);
int genasm_tune_cache_load(genasm_ctx* ctx, const char* path);
int genasm_tune_cache_size(genasm_ctx* ctx);

/*
 * Packs n ASCII bases (host memory) into 2-bit codes (input loading of the
 * candidate pairs of the Results section; host memory, (n+3)/4
 * bytes, layout as for genasm_batch_align_dev). Returns GENASM_E_ALPHABET and
 * sets *bad_index (if not NULL) to the first offending byte.
 */
int genasm_pack(const char* ascii, uint64_t n, uint8_t* packed, uint64_t* bad_index);

/*
 * Device version of genasm_pack (input loading, as genasm_pack), asynchronous
 * on `stream` (NULL = the null stream): packs d_ascii[0..n)
 * into d_packed[0..(n+3)/4) and adds the number of non-ACGT bytes to
 * *d_bad_count (device memory, caller-initialised).
 */
int genasm_pack_dev(genasm_ctx* ctx, const char* d_ascii, uint64_t n, uint8_t* d_packed,
                    uint32_t* d_bad_count, void* stream);

/*
 * Checks arguments of a host-form call without touching a device (library
 * plumbing; the limits are those stated for genasm_batch_align): the values
 * of W, O and k, the offsets (non-decreasing, in range of the given stream
 * lengths) and the alphabet. Returns GENASM_OK or the code genasm_batch_align
 * would return.
 */
int genasm_validate(const char* reads, uint64_t reads_len, const uint64_t* read_off,
                    const char* refs, uint64_t refs_len, const uint64_t* ref_off,
                    uint64_t n_pairs, int32_t k, int32_t W, int32_t O);

/*
 * Profiling of genasm_batch_align_dev calls (off by default); the counters
 * measure what key ideas 1-3 save (Abstract and Introduction: DP-table
 * footprint and accesses). While enabled,
 * each call records HIP events around its stages on the call's stream and
 * fills per-pair work counters; genasm_profile_read waits for the last
 * profiled call and returns its stage times and the counters summed over
 * its pairs. Counters follow the GenASM recurrence: a DC window costs
 * nw * (2 + 6 d*) 64-bit word operations (row 0: shift, or; rows 1..d*:
 * and, shift, or, shift, and, and), the start search n * (2 + 6 d_min).
 */
typedef struct {
    float total_ms;            /* first to last kernel of the call */
    float order_ms;            /* longest-first ordering (batched form) */
    float search_ms;           /* start-search kernels (batched form) */
    float windows_ms;          /* window kernel (batched) or the whole plain kernel */
    uint64_t n_pairs;
    uint64_t window_word_ops;  /* sum of nw * (2 + 6 d*) */
    uint64_t search_word_ops;  /* sum of n * (2 + 6 d_min) */
    uint64_t window_cells;     /* sum over windows of mw * nw */
    uint64_t search_cells;     /* sum of m1 * n */
    uint64_t table_words;      /* sum of (d* + 1) * (min(nw, W-O) + 1): stored DP words */
    uint64_t tb_reads;         /* DP words read by tracebacks */
    uint64_t window_lane_steps;/* lane-steps issued by DC passes, speculative rows included */
    uint64_t search_lane_steps;/* lane-cell-steps issued by the start search */
    uint64_t windows;          /* windows processed */
    uint64_t dc_cycles;        /* shader-clock cycles in DC passes (window setup included), summed over pairs */
    uint64_t tb_cycles;        /* shader-clock cycles in tracebacks and CIGAR stores, summed over pairs */
    uint64_t pair_cycles;      /* shader-clock cycles from a pair's first to last window, summed */
    uint64_t window_workgroups;/* resident workgroups of the batched window kernel (4 groups each) */
} genasm_profile;

/* on: 0 = off; 1 = stage times and the per-pair work counters; 2 = stage
 * times only (the kernels then run exactly as unprofiled, since the counters
 * take registers of their own; genasm_profile_read reports zero counters). */
int genasm_profile_enable(genasm_ctx* ctx, int on);
int genasm_profile_read(genasm_ctx* ctx, genasm_profile* out);
/*
 * Per-pair counters of the last profiled call: GENASM_PROFILE_WORDS uint64
 * words per pair, in pair order: window word ops, search word ops, window
 * cells, search cells, table words, traceback reads, window lane-steps, search
 * lane-steps, windows, DC cycles, traceback cycles, window-loop cycles, and
 * the device's 100 MHz clock when the pair's windows started and ended.
 * *words receives n_pairs * GENASM_PROFILE_WORDS; GENASM_E_NOSPACE (nothing
 * copied) when max_words is smaller.
 */
#define GENASM_PROFILE_WORDS 14
int genasm_profile_pairs(genasm_ctx* ctx, uint64_t* out, uint64_t max_words, uint64_t* words);

/*
 * Serving form: continuous batching of single-pair requests (library
 * plumbing around the same per-pair computation as genasm_batch_align:
 * Introduction, key ideas 1-3 and the traceback step).
 *
 * A server owns an engine thread and device-resident state: a pool of packed
 * read and reference bases, a pool of CIGAR elements, and per-slot window
 * state. Each device iteration (one captured HIP graph):
 *   1. admits waiting requests into free slots while the slot count and both
 *      pools have room (admission by device-memory budget), and runs their
 *      start search;
 *   2. advances every resident pair, the newly admitted ones included, by at
 *      least one window and then until it ends or the iteration's window time
 *      has passed (new pairs and pairs whose last turn was cut short go
 *      first); the window work of all resident pairs overlaps on the device,
 *      and the device itself keeps the lists of unfinished and finished pairs;
 *   3. returns the finished pairs (results, then CIGAR elements) to the host,
 *      which frees their slots and queues their completions.
 * Requests that arrive while others are on the device join at the next
 * iteration; while one iteration runs the engine collects the previous one's
 * output and, with requests waiting, queues the next. A request's result does
 * not depend on the other requests in flight: each pair's windows run exactly
 * as in genasm_batch_align. All requests of one server use its k, W and O.
 */
typedef struct genasm_server genasm_server;

typedef struct {
    int32_t k, W, O;          /* alignment parameters of every request */
    uint32_t max_slots;       /* pairs resident on the device at once; 0 = 32768 */
    uint64_t pool_bases;      /* device pool for resident reads and references, in bases;
                                 0 = 2^29 */
    uint32_t max_pending;     /* requests waiting on the host before genasm_submit returns
                                 GENASM_E_BUSY; 0 = 65536 */
    uint32_t window_budget;   /* windows a resident pair advances per iteration at most;
                                 0 = no limit (the window time alone ends its turn) */
    int32_t use_graph;        /* 1 = replay captured hipGraphs, 0 = launch the kernels
                                 directly; -1 or 0-initialised config: 1 */
    int32_t iteration_us;     /* window time of an iteration in microseconds (fixed);
                                 0 = 2000, and while no request waits and pairs occupy fewer
                                 than half of the window groups a pair's turn also ends from
                                 250 on once a pair of the iteration has finished or a new
                                 request has arrived */
    int32_t cigar_runs;       /* 0 = completions carry CIGAR text; 1 = run-length elements
                                 (GENASM_CIGAR_LEN/OP), as the device form writes them */
    int32_t reserved;
} genasm_server_config;

typedef struct {
    uint64_t tag;             /* the submitter's tag */
    genasm_result result;     /* cigar_off = 0; cigar_len = characters of the text, or
                                 elements with cigar_runs */
    char* cigar;              /* NUL-terminated CIGAR text, or (cigar_runs) an array of
                                 result.cigar_len uint32 elements; owned by the completion */
    uint64_t submit_ns;       /* genasm_now_ns() at submission */
    uint64_t admit_ns;        /* when the request entered a device slot */
    uint64_t done_ns;         /* when its result and CIGAR reached host memory */
} genasm_completion;

typedef struct {
    uint64_t iterations;      /* device iterations run */
    uint64_t submitted, admitted, completed, refused;
    uint32_t resident;        /* requests in device slots now */
    uint32_t pending;         /* requests waiting on the host now */
    uint64_t pool_bases_used;
    double device_ms;         /* summed device time of the iterations (uploads included) */
    uint64_t cancelled;       /* requests cancelled (genasm_cancel) */
} genasm_server_stats;

/* Creates a server on `ctx` (which it then uses exclusively until destroyed).
 * Serving plumbing, as described above. Returns GENASM_E_INVAL for bad
 * parameters, GENASM_E_NOMEM/GENASM_E_DEVICE on allocation or device failure. */
int genasm_server_create(genasm_ctx* ctx, const genasm_server_config* cfg, genasm_server** out);

/* Queues one request (serving plumbing; the pair is aligned as by
 * genasm_batch_align): an ASCII read of m bases and reference of n bases,
 * packed and copied into pinned host memory before return. k, W and O must
 * equal the server's (else GENASM_E_INVAL). Returns GENASM_E_BUSY when
 * max_pending requests already wait, GENASM_E_ALPHABET for a non-ACGT byte,
 * GENASM_E_TOOLONG when the pair can never fit the pools, GENASM_E_NOMEM when
 * no pinned host memory can be had. Thread-safe. */
int genasm_submit(genasm_server* srv, const char* read, uint64_t m, const char* ref, uint64_t n,
                  int32_t k, int32_t W, int32_t O, uint64_t tag);

/* Queues n requests at once (serving plumbing, as genasm_submit) from 2-bit
 * packed host streams (layout as for
 * genasm_batch_align_dev: base b is bits 2*(b%4).. of byte b/4; request i is
 * reads2b bases [read_off[i], read_off[i+1]) against refs2b bases
 * [ref_off[i], ref_off[i+1]), offsets in bases, n + 1 of each), with tags[i].
 * The bases are copied before return. Requests are queued in order while
 * fewer than max_pending wait: *accepted receives how many were queued
 * (requests 0 .. *accepted-1), and the call returns GENASM_E_BUSY when that is
 * fewer than n. GENASM_E_INVAL (nothing queued) for null pointers, decreasing
 * offsets or k/W/O other than the server's, GENASM_E_TOOLONG (nothing queued)
 * when some pair can never fit the pools, GENASM_E_NOMEM (nothing queued) when
 * no pinned host memory can be had. Thread-safe. */
int genasm_submit_batch(genasm_server* srv, const uint8_t* reads2b, const uint64_t* read_off,
                        const uint8_t* refs2b, const uint64_t* ref_off, uint64_t n,
                        int32_t k, int32_t W, int32_t O, const uint64_t* tags,
                        uint64_t* accepted);

/* Moves up to `max` completions into out[] (serving plumbing: each carries the
 * result and CIGAR genasm_batch_align would give its pair), waiting up to
 * timeout_ms for the first one (0 = do not wait); text CIGARs are formatted
 * here, in the calling thread. Returns the number moved, or a negative error (GENASM_E_DEVICE: the
 * engine stopped on a device error). Thread-safe. */
int genasm_poll(genasm_server* srv, genasm_completion* out, int max, int timeout_ms);

/* A completion without its CIGAR, for genasm_poll_batch (64 bytes). */
typedef struct {
    uint64_t tag;
    genasm_result result;     /* cigar_off/cigar_len: run-length elements in the caller's buffer */
    uint64_t submit_ns, admit_ns, done_ns;
} genasm_completion_info;

/* Bulk form of genasm_poll for high-rate consumers (serving plumbing): moves up to `max`
 * completions into out[] and their CIGARs, as run-length elements
 * (GENASM_CIGAR_LEN/OP) in either CIGAR mode, back to back into
 * runs[0 .. runs_cap); result.cigar_off indexes runs. Stops before the first
 * completion whose elements do not fit; *runs_used receives the elements
 * written. Returns the number moved, GENASM_E_NOSPACE when not even the first
 * completion fits (*runs_used then holds the elements it needs), or a
 * negative error as genasm_poll. Thread-safe. */
int genasm_poll_batch(genasm_server* srv, genasm_completion_info* out, int max, uint32_t* runs,
                      uint64_t runs_cap, uint64_t* runs_used, int timeout_ms);

/* Cancels the request with this tag (serving plumbing; the first one found, if tags repeat):
 * a request still waiting on the host is dropped; a resident one runs to its
 * end on the device, then its slot is freed without a completion. Either way
 * no completion for it is delivered. Returns GENASM_E_INVAL when no waiting
 * or resident request has the tag (already completed, or never submitted).
 * Thread-safe. */
int genasm_cancel(genasm_server* srv, uint64_t tag);

/* Frees the CIGAR of a completion (serving plumbing). Safe on NULL. */
void genasm_completion_release(genasm_completion* c);

/* Copies the server's counters (serving plumbing). GENASM_E_INVAL for NULL. */
int genasm_server_stats_read(genasm_server* srv, genasm_server_stats* out);

/* Stops the engine (requests still waiting are dropped; iterations on the
 * device complete first) and frees the server (serving plumbing). Safe on NULL. */
void genasm_server_destroy(genasm_server* srv);

/* Monotonic clock used by the completion timestamps, in nanoseconds (serving
 * plumbing). */
uint64_t genasm_now_ns(void);

/*
 * Measured limits of the device the context runs on (library plumbing: the
 * denominators of the roofline the window kernel is reported against; no
 * paper passage). Each is the rate of a microbenchmark with exactly known
 * work, timed with HIP events on the context's stream:
 *   dc_mix_tops  the DC recurrence's own step in registers, as the window
 *                kernels execute it (one DPP lane shift of a 64-bit word and
 *                six 64-bit and/or/shift operations worked on 32-bit halves,
 *                counted as 12 int32 operations), on independent chains at
 *                full occupancy;
 *   int32_tops   plain 32-bit and/or/xor chains;
 *   lds_tbps     16-byte LDS reads without bank conflicts;
 *   hbm_tbps     a 1 GiB device-to-device copy (read + write bytes);
 *   shift64_tops v_lshlrev_b64 chains (each counted as two int32 operations);
 *   funnel_tops  v_alignbit_b32 chains (32-bit funnel shift);
 *   dpp_tops     v_mov_b32_dpp row rotations.
 * Allocates about 2 GiB of device memory for the duration of the call.
 */
typedef struct {
    double dc_mix_tops;   /* int32 lane-operations per second / 1e12 */
    double int32_tops;
    double lds_tbps;      /* bytes per second / 1e12 */
    double hbm_tbps;
    double shift64_tops;  /* int32 lane-operations per second / 1e12 */
    double funnel_tops;
    double dpp_tops;
    int32_t compute_units;
    int32_t reserved;
} genasm_peaks;
int genasm_measure_peaks(genasm_ctx* ctx, genasm_peaks* out);

/* Library version string (library plumbing). */
const char* genasm_version(void);

#ifdef __cplusplus
}
#endif

#endif /* GENASM_H */
