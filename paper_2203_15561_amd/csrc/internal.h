// Internal interface between the host runtime and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <string>

#include "genasm.h"

// Library context (opaque in the C ABI).
struct genasm_ctx {
    int device = -1;
    hipStream_t stream = nullptr;
    int num_cus = 0;
    std::string err;
    // device scratch arena
    char* scratch = nullptr;
    size_t scratch_cap = 0;
    // bit planes of the current call's streams (device)
    char* planes = nullptr;
    size_t planes_cap = 0;
    // unimproved-form window tables (device)
    char* unimp = nullptr;
    size_t unimp_cap = 0;
    // host-form staging (device)
    char* stage = nullptr;
    size_t stage_cap = 0;
    // debug builds: per-pair audit words (device)
    char* dbg = nullptr;
    size_t dbg_cap = 0;
    // device address of the static scratch of the no-allocation device form
    // on this context's device
    void* static_scratch = nullptr;
    // set by a device-form call made under stream capture: a graph may hold
    // raw pointers into the buffers above, so they must not be freed or moved
    // until genasm_unpin
    bool pinned = false;
    // profiling
    bool profiling = false;      // stage times (HIP events) of device-form calls
    bool prof_counters = false;  // and the per-pair work counters
    bool have_profile = false;
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    char* stats = nullptr;
    size_t stats_cap = 0;
    uint64_t prof_pairs = 0;
    int prof_form = 0;
    int prof_window_blocks = 0;
    // autotuner cache: workload signature -> fastest launch and its time
    struct Tuned {
        genasm_launch launch;
        float ms;
    };
    std::map<std::string, Tuned> tune;
};

namespace genasm {

// Resumable per-pair window state (serving: pairs advance a few windows per
// iteration and keep their state in device memory between iterations).
struct PairState {
    int32_t ti, pj;       // reference / read cursor
    int32_t score;        // committed edits
    uint32_t nwin;        // windows processed
    uint32_t written;     // CIGAR elements already in device memory
    int32_t cur_op;       // op of the open CIGAR run, -1 before the first op
    uint32_t cur_len;
    uint32_t flags;       // kState* bits
};
constexpr uint32_t kStateStarted = 1u;
constexpr uint32_t kStateDone = 2u;       // result written
constexpr uint32_t kStateFailed = 4u;
constexpr uint32_t kStateInternal = 8u;
constexpr uint32_t kStateOverflow = 16u;
constexpr uint32_t kStateDeep = 32u;      // compact groups: the last window needed 16 rows or more

// Per-pair start-search outcome kept in device scratch.
struct SearchOut {
    int32_t row;   // least edit row with a hit; kSearchFailed / kSearchDone when no window work
    uint32_t col;  // leftmost hit column of that row
};
constexpr int32_t kSearchFailed = -1;  // no hit within K rows: the result is already written
constexpr int32_t kSearchDone = -2;    // empty read: the result is already written
constexpr int32_t kSearchPending = -3; // not searched yet (retry list)

// Turn limits of a serving iteration (device wall clock, 100 MHz), written at
// its start. A resident pair's turn takes at least one window and starts none
// at or past `end`; from `soon` on it also ends once a pair of the iteration
// has finished or the host has counted more arrivals than `admitted`.
struct TurnLimits {
    unsigned long long end, soon, admitted;
};

struct AlignParams {
    const uint8_t* reads;       // 2-bit packed read stream
    const uint64_t* read_off;   // n_pairs + 1 base offsets
    const uint8_t* refs;        // 2-bit packed reference stream
    const uint64_t* ref_off;
    // The same streams as bit planes (see launch_planes), read by the window
    // kernels. Word w of a plane holds bit 0 (lo) or bit 1 (hi) of the codes of
    // bases origin + 64w .. origin + 64w + 63, where origin is read_off[0]
    // (ref_off[0]) rounded down to a multiple of 64 when planes_from_off0 is
    // set, else 0.
    const unsigned long long* read_lo;
    const unsigned long long* read_hi;
    const unsigned long long* ref_lo;
    const unsigned long long* ref_hi;
    int32_t planes_from_off0;
    uint64_t n_pairs;
    int32_t K;                  // min(k, W)
    int32_t W;
    int32_t L;                  // W - O: bases committed per window at most
    int32_t stride;             // words per stored table row: L + 2 (see kernels.hip, OFF_TAB)
    genasm_result* out;
    uint32_t* cigar;            // CIGAR elements
    uint64_t cigar_cap;
    SearchOut* search;          // per pair
    const uint32_t* order;      // window-kernel pair order (null = identity)
    uint32_t* counters;         // device queue heads and list lengths (see kCounter*)
    const uint32_t* list_in;    // search items / finalize: pairs to search (null = all pairs)
    uint32_t* list_out;         // (unused)
    const uint64_t* items_in;   // search stage: (pair << 24 | chunk) items to search
    uint64_t* items_out;        // search: items for the next stage (or stage 0, from k_search_items)
    unsigned long long* search_key;  // per pair: least (row << 32 | column) hit found so far
    uint32_t search_chunk;      // reference columns per search item (0 = whole reference)
    unsigned long long* spill;  // window table rows >= lds_rows, per worker
    int32_t lds_rows;
    int32_t list_slot;          // which counters[] pair this search stage uses
    unsigned long long* stats;  // optional, kStatCount counters per pair (null = off)
    uint32_t* easy_list;        // pairs for the 16-lane window groups (filled by the search)
    uint32_t* hard_list;        // pairs for whole-wavefront windows (start row >= hard_row)
    int32_t hard_row;
    int32_t hard_lanes;         // lanes per pair for the hard list: 16, 32 (two pairs per wavefront) or 64
    int32_t tb_prefetch;        // tracebacks over spilled rows load the next row ahead
    int32_t hard_share;         // percent of window workers that start on the hard queue
    int32_t route;              // search: append finished pairs to the window lists
    int32_t compact;            // window kernel: compact 16-lane groups (32-bit table slices)
    // Optional per-pair layout (serving: sequences sit anywhere in a device pool).
    const uint32_t* read_len;   // if set, pair i's read is [read_off[i], read_off[i] + read_len[i])
    const uint32_t* ref_len;
    const uint64_t* run_base;   // if set, first CIGAR element of pair i; else from the offsets
    PairState* state;           // if set, window state persists here between launches
    uint32_t window_budget;     // windows a pair may advance per launch (0 = to the end)
    // Serving iterations (all null outside the serving form):
    const TurnLimits* turn;     // when a resident pair's turn in this launch ends
    const unsigned long long* arrivals;  // requests the host has counted so far (device word)
    uint32_t* fin_list;         // pairs that ended in this launch (their result is written)
    uint32_t* fin_len;
    uint32_t* next_hot;         // unfinished pairs that advanced at most one window
    uint32_t* next_cold;        // unfinished pairs that advanced more
    uint32_t* next_len;         // counters block of the next launch: its easy (hot) and hard
                                // (cold) list lengths at kCounterEasyLen / kCounterHardLen
    // Debug builds (GENASM_DEBUG) only: per-pair audit word (kAudit* bits in the
    // low half, the number of workers that took the pair in the high half).
    uint32_t* audit;
};

// Audit bits of a debug build: an invariant that failed for the pair. The
// check runs before the access it guards, and a failed check ends the pair
// (GENASM_FLAG_INTERNAL) instead of letting the access go out of bounds.
constexpr uint32_t kAuditWindow = 1u;  // window sizes outside 1..W, or W past 64
constexpr uint32_t kAuditLds = 2u;     // a DC pass's rows or columns outside the LDS table
constexpr uint32_t kAuditSpill = 4u;   // a DC pass's rows outside the worker's spill area
constexpr uint32_t kAuditRuns = 8u;    // more run records than the run area holds
constexpr uint32_t kAuditTable = 16u;  // a traceback read outside the rows or columns stored
constexpr uint32_t kAuditQueue = 32u;  // a pair taken by no window worker or by more than one
constexpr uint32_t kAuditTake = 1u << 16;  // one worker took the pair

// Per-pair work counters written when AlignParams::stats is set.
constexpr int kStatWindowWordOps = 0;   // sum over windows of nw * (2 + 6 d*)  (64-bit DC ops)
constexpr int kStatSearchWordOps = 1;   // n * (2 + 6 d_min)
constexpr int kStatWindowCells = 2;     // sum over windows of mw * nw
constexpr int kStatSearchCells = 3;     // m1 * n
constexpr int kStatTableWords = 4;      // sum over windows of (d* + 1) * (min(nw, W-O) + 1)
constexpr int kStatTbReads = 5;         // table words read by traceback
constexpr int kStatWindowLaneSteps = 6; // lane-steps issued by DC passes (speculative rows included)
constexpr int kStatSearchLaneSteps = 7; // lane-steps issued by the start search (all stages)
constexpr int kStatWindows = 8;         // windows processed
constexpr int kStatDcCycles = 9;        // shader-clock cycles: window setup and DC passes
constexpr int kStatTbCycles = 10;       // shader-clock cycles: traceback and run stores
constexpr int kStatPairCycles = 11;     // shader-clock cycles of the pair's window loop
constexpr int kStatPairStart = 12;      // device clock (100 MHz) when the pair's windows started
constexpr int kStatPairEnd = 13;        // device clock (100 MHz) when they ended
constexpr int kStatCount = 14;

// counters[] layout: queue heads and list lengths for the batched pipeline.
constexpr int kCounterListBase = 2;  // search stage s: counters[2 + 2s] = list length, [3 + 2s] = head
constexpr int kCounterEasyLen = 10;
constexpr int kCounterEasyHead = 11;
constexpr int kCounterHardLen = 12;
constexpr int kCounterHardHead = 13;
constexpr int kCounterPairs = 14;    // pairs the search items / finalize kernels walk
constexpr int kCounterCount = 16;

// LDS words per group, by kernel.
constexpr int kGroupHeaderWords = 158;   // window groups: PM columns, boundary row, broadcast
// A window group: header, lds_rows table rows, one end word (the last row's
// right dummy slot).
__host__ __device__ inline int window_group_words(int lds_rows, int stride) {
    return kGroupHeaderWords + lds_rows * stride + 1;
}
// 32-lane window groups have a longer header (their PM column and boundary
// arrays each span 31 more words).
constexpr int kGroupHeaderWords32 = 192;
__host__ __device__ inline int window_group_words32(int lds_rows, int stride) {
    return kGroupHeaderWords32 + lds_rows * stride + 1;
}
// Compact window groups keep every row of a deep window in their spill area.
constexpr int kCompactSpillRows = 64;
// Spilled table rows are kept in step order: each spilled pass of a G-lane
// group is a block of 64 + G slots of G words (the entry lane g computes at
// step t sits at slot t + 1, word (t + 1) G + g), so the G stores of a step
// fill adjacent words.
__host__ __device__ constexpr int spill_pass_words(int G) { return (64 + G) * G; }
// Words of one 16-lane group's spill area for `spill_rows` spilled rows (a
// multiple of 16): one block per spilled pass, and at least half a 32-lane
// block, since a 32-lane group keeps its spilled pass in the areas of the two
// 16-lane groups it replaces.
__host__ __device__ inline int spill_group_words(int spill_rows) {
    if (spill_rows <= 0) return 0;
    const int passes = spill_rows / 16 * spill_pass_words(16);
    const int half32 = spill_pass_words(32) / 2;
    return passes > half32 ? passes : half32;
}
// Words of the spill of `workers` 16-lane groups and an end word.
inline uint64_t spill_words(uint64_t workers, int spill_rows) {
    return workers * (uint64_t)spill_group_words(spill_rows) + 1;
}
// Start search group: PM and broadcast slots, then a ring of 128 text masks
// kept twice (words kSearchRingOff + w and + 128 + w).
constexpr int kSearchRingOff = 160;
constexpr int kSearchGroupWords = kSearchRingOff + 256;

// Kernel launchers (kernels.hip). All return hipError_t of the launch.
hipError_t launch_plain(const AlignParams& p, hipStream_t s);
// Pre-alignment filter: dist[i] = least edit distance of read i against any
// substring of reference i when <= k (k <= 63), else -1; start[i] = leftmost
// start of such a substring. Reads up to 1024 bases (filter_words gives the
// 64-bit words per row; 0 = too long).
int filter_words(uint32_t max_read_len);
hipError_t launch_filter(const uint8_t* reads, const uint64_t* read_off, const uint8_t* refs,
                         const uint64_t* ref_off, uint64_t n_pairs, uint32_t max_read_len,
                         int32_t k, int32_t* dist, uint32_t* start, hipStream_t s);
// Unimproved form (ablation): one pair per workgroup, its window table (all
// rows, four edge words per entry) in `table`, unimproved_table_words(n_pairs)
// words of device memory.
uint64_t unimproved_table_words(uint64_t n_pairs);
hipError_t launch_unimproved(const AlignParams& p, unsigned long long* table, hipStream_t s);
hipError_t launch_search(const AlignParams& p, int group_lanes, int rows_per_lane, int blocks,
                         hipStream_t s);
// Start-search workgroups one compute unit holds at once, 0 on error.
int search_blocks_per_cu(int group_lanes, int rows_per_lane);
hipError_t launch_windows(const AlignParams& p, int blocks, hipStream_t s);
// Debug builds: after the window kernel, checks that every pair whose search
// hit was taken by exactly one worker (batched form: `queued` = 1) and marks
// each pair with an audit bit GENASM_FLAG_INTERNAL in its result.
hipError_t launch_audit(const AlignParams& p, int queued, hipStream_t s);
// Window workgroups one compute unit holds at once (registers and LDS), 0 on error.
int windows_blocks_per_cu(const AlignParams& p);
hipError_t launch_pack(const char* ascii, uint64_t n, uint8_t* packed, uint32_t* bad,
                       hipStream_t s);
hipError_t launch_init_counters(uint32_t* counters, uint32_t n_pairs, hipStream_t s);
// Start search: stage-0 items of the listed pairs (list_in, count in
// counters[kCounterPairs]; all pairs when list_in is null), the stages, then
// the per-pair outcome and window routing.
hipError_t launch_search_items(const AlignParams& p, uint32_t max_pairs, hipStream_t s);
hipError_t launch_search_finalize(const AlignParams& p, uint32_t max_pairs, hipStream_t s);
// Reference columns per start-search item: batched calls and the serving loop.
constexpr uint32_t kBatchSearchChunk = 4096;
constexpr uint32_t kServeSearchChunk = 1024;
// Upper bound of the search items of a batch.
inline uint64_t search_item_cap(uint64_t n_pairs, uint64_t total_ref_bases, uint32_t chunk) {
    return chunk ? n_pairs + total_ref_bases / chunk + 1 : n_pairs + 1;
}
// Serving iterations. A device parameter block (copied from the host before
// each launch or graph replay) holds kServeParam* words.
constexpr int kServeParamNew = 0;       // pairs admitted in this iteration
constexpr int kServeParamTicks = 1;     // window time of the iteration, 100 MHz ticks (0 = none)
constexpr int kServeParamSoonTicks = 2; // from then on the turn also ends on news (0 = at the end)
constexpr int kServeParamAdmitted = 3;  // arrivals admitted so far (low word; high word at 4)
constexpr int kServeParamWords = 8;
// One admitted request: its slot and where its bases and CIGAR go in the pools.
struct ServeAdmit {
    uint64_t read_off, ref_off, run_base;
    uint32_t slot, m, n, pad;
};
// Per-slot tables the admission kernel fills.
struct ServeSlots {
    uint64_t* read_off;
    uint64_t* ref_off;
    uint64_t* run_base;
    uint32_t* read_len;
    uint32_t* ref_len;
    PairState* state;
};
// Starts an iteration: clears the search and queue counters of this
// iteration's block `cur` (kCounterPairs = admitted pairs), the next block's
// list lengths and the finished count, then writes the admitted slots'
// tables, resets their window state and lists them in new_list.
hipError_t launch_serve_begin(uint32_t* cur, uint32_t* next, uint32_t* fin_len,
                              const uint32_t* params, const ServeAdmit* admit, ServeSlots slots,
                              uint32_t* new_list, hipStream_t s);
// Writes the iteration's turn limits from the parameter block and the device clock.
hipError_t launch_serve_stamp(const uint32_t* params, TurnLimits* turn, hipStream_t s);
// Ends an iteration: the finished pairs' CIGAR offsets (a prefix sum over
// their element counts) into fin_off, their slots and results (cigar_off =
// that offset) into the host-mapped summary (hdr[0] = count, hdr[1] = total
// elements), then their CIGAR elements from the pool into dst (elements past
// dst_cap are left for the host to fetch).
hipError_t launch_serve_finish(const uint32_t* fin_list, const uint32_t* fin_len,
                               const genasm_result* out, uint64_t* fin_off,
                               unsigned long long* hdr, uint32_t* sum_slot,
                               genasm_result* sum_res, const uint32_t* cigar, uint32_t* dst,
                               uint64_t dst_cap, uint32_t max_fin, hipStream_t s);
hipError_t launch_fill_u64(unsigned long long* p, uint64_t n, unsigned long long v, hipStream_t s);
// Longest-read-first pair order (approximate: reads are bucketed by length)
// into order[0..n_pairs); hist is kLptBuckets words of scratch.
constexpr int kLptBuckets = 336;
// Clears n 32-bit words.
hipError_t launch_zero_u32(uint32_t* p, uint64_t n, hipStream_t s);
hipError_t launch_lpt_order(const uint64_t* read_off, uint64_t n_pairs, uint32_t* hist,
                            uint32_t* order, hipStream_t s);
hipError_t launch_compact_cigar(const genasm_result* d_out, const uint64_t* dst_off,
                                uint64_t n_pairs, const uint32_t* cigar, uint32_t* dst,
                                hipStream_t s);

// Scatters byte ranges: for k < n, copies len[k] bytes from src + src_off[k]
// to dst + dst_off[k] (serving: packed sequences into the device pool).
hipError_t launch_scatter_bytes(const uint8_t* src, const uint64_t* src_off, uint8_t* dst,
                                const uint64_t* dst_off, const uint32_t* len, uint32_t n,
                                hipStream_t s);

// Bit planes of bases [b0, b0 + n_bases) of a 2-bit packed stream, where b0 =
// *d_first (device memory; 0 if d_first is null): with origin = b0 rounded
// down to a multiple of 64, lo[w] / hi[w] bit k is bit 0 / bit 1 of the code
// of base origin + 64w + k (0 past b0 + n_bases). Writes plane_words(n_bases)
// words per plane; the last words are padding that the window kernels may
// read ahead into.
inline uint64_t plane_words(uint64_t n_bases) { return (n_bases + 63 + 63) / 64 + 3; }
hipError_t launch_planes(const uint8_t* packed, const uint64_t* d_first, uint64_t n_bases,
                         unsigned long long* lo, unsigned long long* hi, hipStream_t s);
// Serving: converts n uploaded ranges of packed bases (range k: len[k] bases
// at byte src_off[k] of src) into the plane pool at word dst_word[k] (ranges
// start on a 64-base boundary).
hipError_t launch_scatter_planes(const uint8_t* src, const uint64_t* src_off, const uint32_t* len,
                                 unsigned long long* lo, unsigned long long* hi,
                                 const uint64_t* dst_word, uint32_t n, hipStream_t s);

// Occupancy helpers.
int plain_lds_bytes(int stride);
int window_lds_bytes(int lds_rows, int stride);
int compact_lds_bytes(int stride);
int search_lds_bytes(int group_lanes);

}  // namespace genasm
