// gfx950 kernels of the GenASM aligner: 2-bit packing, start search, windowed
// DC + TB with the paper's three improvements (Introduction, key ideas 1-3),
// and CIGAR compaction.
//
// Work decomposition. A "group" is G consecutive lanes of a 64-lane wavefront
// (G = 16 or 64) that handles one (read, reference) pair at a time. Lane gl
// of the group owns DP row d = c*G + gl in pass c, and the G rows advance as an
// anti-diagonal wavefront over the text columns: at step t lane gl computes
// column i = nw-1-t+gl, so the row above (lane gl-1) produced column i one step
// earlier and hands it over with a one-lane DPP shift (row_shr:1 inside a
// 16-lane row, wave_shr:1 across the whole wavefront). Each cell is
//   R[d][i] = D & (((D & U) << 1) | [d == 0]) & ((R[d][i+1] << 1) | PM[T[i]])
// with D = R[d-1][i+1] and U = R[d-1][i]; this is the AND of the match,
// substitution, insertion and deletion bitvectors of the GenASM recurrence,
// folded into four 64-bit operations.
//
// Improvement 1: only R (the AND) is stored per entry. Improvement 2: rows are
// computed G at a time and no further pass runs once a row's column 0 has its
// top bit clear. Improvement 3: only columns 0..min(nw, W-O) are stored, the
// only ones the traceback of a window can reach; rows at or above the read
// window length are never stored at all (their used bits are all zero).
// The stored table lives in LDS; rows past `lds_rows` spill to device memory.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "internal.h"

namespace genasm {

typedef unsigned long long u64;

// ---------------------------------------------------------------------------
// Small device helpers
// ---------------------------------------------------------------------------

__device__ __forceinline__ u64 init_word(int d) { return d >= 64 ? 0ull : (~0ull << d); }

__device__ __forceinline__ int clampi(int x, int lo, int hi) { return min(max(x, lo), hi); }

// min(max(x, lo), hi) in one v_med3_i32 (lo <= hi).
__device__ __forceinline__ int med3i(int x, int lo, int hi) {
#if defined(__HIP_DEVICE_COMPILE__)
    int r;
    asm("v_med3_i32 %0, %1, %2, %3" : "=v"(r) : "v"(x), "v"(lo), "v"(hi));
    return r;
#else
    return min(max(x, lo), hi);
#endif
}

// Shift a 64-bit value by one lane with a DPP move; lanes without a source lane
// inside their DPP row (or the wavefront, for wave_shr) receive `old`.
template <int CTRL>
__device__ __forceinline__ u64 dpp64(u64 old, u64 src) {
    const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp((int)(unsigned)old, (int)(unsigned)src,
                                                              CTRL, 0xF, 0xF, false);
    const unsigned hi = (unsigned)__builtin_amdgcn_update_dpp((int)(unsigned)(old >> 32),
                                                              (int)(unsigned)(src >> 32), CTRL, 0xF,
                                                              0xF, false);
    return ((u64)hi << 32) | lo;
}

constexpr int kDppRowShr1 = 0x111;
constexpr int kDppRowRor1 = 0x121;
constexpr int kDppWaveShr1 = 0x138;
constexpr int kDppWaveRor1 = 0x13C;

template <int G> struct LaneShift;
// A rotation writes every lane, so it needs no `old` value (and no copy of the
// source into the destination first).
template <int CTRL>
__device__ __forceinline__ u64 dpp64_rot(u64 src) {
    const unsigned lo = (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)src, CTRL, 0xF, 0xF, false);
    const unsigned hi = (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)(src >> 32), CTRL, 0xF,
                                                           0xF, false);
    return ((u64)hi << 32) | lo;
}

template <> struct LaneShift<16> {
    // value of lane gl-1 within the 16-lane group; lane 0 gets `old`
    static __device__ __forceinline__ u64 up(u64 old, u64 v) { return dpp64<kDppRowShr1>(old, v); }
    // value of lane gl-1, lane 0 gets lane 15 (rotation inside the group)
    static __device__ __forceinline__ u64 rot(u64 v) { return dpp64_rot<kDppRowRor1>(v); }
};
template <> struct LaneShift<64> {
    static __device__ __forceinline__ u64 up(u64 old, u64 v) { return dpp64<kDppWaveShr1>(old, v); }
    static __device__ __forceinline__ u64 rot(u64 v) { return dpp64_rot<kDppWaveRor1>(v); }
};
// Two 32-lane groups per wavefront: a shift over the whole wavefront, after
// which lane 32 holds lane 31's value; shift_up gives it `old` instead.
template <> struct LaneShift<32> {
    static __device__ __forceinline__ u64 up(u64 old, u64 v) { return dpp64<kDppWaveShr1>(old, v); }
};

// Value of lane gl-1 of the group; lane 0 of the group gets `old`.
template <int G>
__device__ __forceinline__ u64 shift_up(u64 old, u64 v, int gl) {
    const u64 s = LaneShift<G>::up(old, v);
    if constexpr (G == 32) return gl == 0 ? old : s;
    return s;
}

// Orders the LDS accesses of one wavefront: the compiler may not move memory
// operations across it, and it waits for the wavefront's outstanding LDS
// operations (LDS executes one wavefront's operations in order). This holds for
// DS instructions only, so the kernels must reach a group's LDS through
// pointers the compiler knows to be LDS: an out-of-line callee would get
// generic pointers and FLAT accesses. The per-pair functions are forced
// inline, and tests/test_kernel_asm.py checks that the kernels make no calls.
// s_waitcnt immediates (gfx9 encoding): lgkmcnt(0) alone, and vmcnt(0) lgkmcnt(0).
constexpr int kWaitLgkm0 = 0xC07F;
constexpr int kWaitVm0Lgkm0 = 0x0070;

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_s_waitcnt(kWaitLgkm0);
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// As wave_sync, and also waits for the wavefront's device-memory accesses.
__device__ __forceinline__ void mem_sync() {
    __builtin_amdgcn_s_waitcnt(kWaitVm0Lgkm0);
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ int base_at(const uint8_t* s, uint64_t b) {
    return (s[b >> 2] >> ((unsigned)(b & 3) * 2)) & 3;
}

__device__ __forceinline__ u64 pick_pm(u64 p0, u64 p1, u64 p2, u64 p3, int c) {
    const u64 lo = (c & 1) ? p1 : p0;
    const u64 hi = (c & 1) ? p3 : p2;
    return (c & 2) ? hi : lo;
}

__device__ __forceinline__ u64 group_ballot(bool pred, int G, int lane) {
    const u64 b = __ballot(pred);
    if (G == 64) return b;
    const int shift = lane & ~(G - 1);
    return (b >> shift) & ((1ull << G) - 1);
}

// Loads of a group's spilled table rows. The rows are written and read back by
// the same wavefront, so wavefront scope is enough (a device-scope load would
// skip the XCD's L2 for data that never leaves this CU).
__device__ __forceinline__ u64 load_spill(const u64* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
}

// Entry (row r, column col) of a window's spilled rows (r >= lds_rows, a
// multiple of G): the rows are kept in step order, one block of
// spill_pass_words(G) per spilled pass, lane g = (r - lds_rows) mod G of the
// pass holding column col at slot nw - col + g (the slot of the step that
// computed it, plus one). Slots below 0 (columns past nw + g, which no step
// computes and whose values a reader does not use) read slot 0.
template <int G>
__device__ __forceinline__ const u64* spill_entry(const u64* spill, int r, int col, int nw,
                                                  int lds_rows) {
    const int q = r - lds_rows;
    const int g = q & (G - 1);
    const int slot = max(nw - col + g, 0);
    return spill + (size_t)(q / G) * spill_pass_words(G) + slot * G + g;
}

// Per-group LDS layout (64-bit words).
constexpr int OFF_PM = 0;      // 4 pattern masks / match accumulators
constexpr int OFF_PMT = 4;     // PM[T[i]] for i in 0..nw, ~0 at nw..64 (66 words)
constexpr int OFF_BROW = 70;   // boundary row between passes: slot 1+i, i in -1..nw+1 (68 words)
constexpr int OFF_CH = 138;    // 64 pattern bytes, 64 text bytes (16 words)
constexpr int OFF_BC = 154;    // broadcast slots (4 words)
// Stored table rows, `stride` = W-O+2 words each: slot 0 and slot W-O+2 are
// dummies that absorb the stores of steps outside columns 0..W-O; the right
// dummy of row r is the left dummy of row r+1 (both only ever hold garbage),
// and the group's last row has an end word of its own.
constexpr int OFF_TAB = 158;
static_assert(OFF_TAB == kGroupHeaderWords, "layout");
static_assert(OFF_BC + 4 <= kSearchRingOff, "layout");

// Layout of a 16-lane window group (in step order, so that a DC step needs no
// address arithmetic): PMT16[x] = PM[T[nw-1-x]] at word OFF_PMT16 + x for
// x in -15..63 (~0 below 0 and from nw on); BROW16[z] = the pass's last row at
// column nw-1-z at word OFF_BROW16 + z, written for z from -15 on (by lane 15,
// for the columns past the stored range; the others are copied from the table
// row before a next pass) and read for z in 0..nw+29 (the operand loads run U
// steps ahead of whole U-step chunks). Lane g at step t reads PMT16[t-g]; lane
// 0 reads BROW16[t]; lane 15 writes BROW16[t-15]. The regions nobody needs
// overlap: PMT16 past
// x = 63 (read only by finished lanes) with BROW16 below z = 0 (written only
// by lanes ahead of the text), and BROW16 past z = 63 (read only by finished
// lanes) with the broadcast slots and the first table row.
constexpr int OFF_PMT16 = 15;
constexpr int OFF_BROW16 = 94;
constexpr int OFF_RUNS16 = OFF_BROW16;  // traceback run records (the DC arrays are dead then)
static_assert(OFF_PMT16 + 64 + 15 == OFF_BROW16, "layout");

// The same step-ordered layout for G-lane groups (G = 16 or 32): PMT at word
// G-1+x for x in -(G-1)..64, BROW at word 2(G-1)+64+z, written for z in
// -(G-1)..nw-1 and read for z in 0..nw+G+13, the table after the header. The
// 32-lane header ends past BROW[63] (word 189); the reads past it go into the
// first table row, and the broadcast slot lies inside BROW (group_pop uses it
// only between pairs). Run records go at OFF_BROW16 (16 lanes) or OFF_BROW
// (words 70..133 at most: at most 2 min(L, d*) + 1 <= 127 runs of 32 bits).
template <int G> struct SoLayout {
    static_assert(G == 16 || G == 32, "step-ordered layout: 16 or 32 lanes");
    static constexpr int pmt = G - 1;
    static constexpr int brow = 2 * (G - 1) + 64;
    static constexpr int tab = G == 16 ? kGroupHeaderWords : kGroupHeaderWords32;
};
static_assert(SoLayout<16>::pmt == OFF_PMT16 && SoLayout<16>::brow == OFF_BROW16 &&
              SoLayout<16>::tab == OFF_TAB, "layout");
static_assert(SoLayout<32>::brow + 64 <= kGroupHeaderWords32, "layout");
static_assert(OFF_BROW + 64 <= SoLayout<32>::tab, "layout");

// First table word and run-record word of a G-lane group.
template <int G> constexpr int tab_off() { return G == 32 ? kGroupHeaderWords32 : OFF_TAB; }
template <int G> constexpr int runs_off() { return G == 16 ? OFF_RUNS16 : OFF_BROW; }

// ---------------------------------------------------------------------------
// Pattern masks
// ---------------------------------------------------------------------------

// Builds PM for pattern bases P[0..mw) (read stream offset rb) into
// lds[OFF_PM..+4): bit q of PM[c] is 0 iff P[mw-1-q] == c. Also stores the
// pattern bases as bytes at OFF_CH when `keep_chars`.
template <int G>
__device__ void build_pm(u64* lds, int gl, const uint8_t* reads, uint64_t rb, int mw,
                         bool keep_chars) {
    uint8_t* pch = reinterpret_cast<uint8_t*>(lds + OFF_CH);
    u64* acc = lds + OFF_PM;
    if (gl < 4) acc[gl] = 0ull;
    wave_sync();
#pragma unroll
    for (int u = 0; u < 64 / G; ++u) {
        const int b = gl + u * G;
        const int c = b < mw ? base_at(reads, rb + b) : 0;
        if (keep_chars) pch[b] = (uint8_t)c;
        if (b < mw) atomicOr(&acc[c], 1ull << (mw - 1 - b));
    }
    wave_sync();
    if (gl < 4) acc[gl] = ~acc[gl];
    wave_sync();
}

// One DC step on a 64-bit word: R' = x & ((R << 1) | pm) with
// x = D & (((D & up) << 1) | low), worked on 32-bit halves: the low half's
// shift and OR are one instruction and the high half's shift is a funnel shift,
// which together issue faster on gfx950 than the 64-bit shift instruction.
__device__ __forceinline__ u64 dc_step(u64 R, u64 D, u64 up, u64 pm, u64 low) {
    const uint32_t Rl = (uint32_t)R, Rh = (uint32_t)(R >> 32);
    const uint32_t Dl = (uint32_t)D, Dh = (uint32_t)(D >> 32);
    const uint32_t el = Dl & (uint32_t)up, eh = Dh & (uint32_t)(up >> 32);
    const uint32_t xl = Dl & ((el << 1) | (uint32_t)low);
    const uint32_t xh = Dh & (__builtin_amdgcn_alignbit(eh, el, 31) | (uint32_t)(low >> 32));
    const uint32_t sl = (Rl << 1) | (uint32_t)pm;
    const uint32_t sh = __builtin_amdgcn_alignbit(Rh, Rl, 31) | (uint32_t)(pm >> 32);
    return ((u64)(xh & sh) << 32) | (xl & sl);
}

// Bits 0, 2, 4, .. of w into the low half and bits 1, 3, 5, .. into the high
// half (bit 2k to bit k, bit 2k+1 to bit 32+k).
__device__ __forceinline__ u64 split_even_odd(u64 w) {
    auto compress = [](u64 x) -> u64 {
        x &= 0x5555555555555555ull;
        x = (x | (x >> 1)) & 0x3333333333333333ull;
        x = (x | (x >> 2)) & 0x0F0F0F0F0F0F0F0Full;
        x = (x | (x >> 4)) & 0x00FF00FF00FF00FFull;
        x = (x | (x >> 8)) & 0x0000FFFF0000FFFFull;
        return (x | (x >> 16)) & 0x00000000FFFFFFFFull;
    };
    return compress(w) | (compress(w >> 1) << 32);
}

// Shifts a two-word bit window: bits [s, s+64) of the 128-bit value (hi:lo).
__device__ __forceinline__ u64 funnel64(u64 lo, u64 hi, int s) {
    return s == 0 ? lo : (lo >> s) | (hi << (64 - s));
}

// Read-ahead cursor over the two bit planes of one sequence: words q, q+1, q+2
// of each plane. A window needs the 64 bits starting at some bit of word q;
// the next window starts at most 64 bases later, so it needs at most word
// q+2, whose load was issued one window earlier.
struct SeqCursor {
    u64 lo0, lo1, lo2, hi0, hi1, hi2;
    uint64_t q;
};

__device__ __forceinline__ void seq_open(SeqCursor& c, const u64* lo, const u64* hi, uint64_t bit) {
    c.q = bit >> 6;
    c.lo0 = lo[c.q]; c.lo1 = lo[c.q + 1]; c.lo2 = lo[c.q + 2];
    c.hi0 = hi[c.q]; c.hi1 = hi[c.q + 1]; c.hi2 = hi[c.q + 2];
}

// Moves the cursor to the window starting at `bit` (at most one word on) and
// returns that window's 64 bases as (lo, hi) planes: bit k = base bit + k.
__device__ __forceinline__ void seq_window(SeqCursor& c, const u64* lo, const u64* hi,
                                           uint64_t bit, u64& wlo, u64& whi) {
    if ((bit >> 6) != c.q) {
        c.q += 1;
        c.lo0 = c.lo1; c.lo1 = c.lo2; c.lo2 = lo[c.q + 2];
        c.hi0 = c.hi1; c.hi1 = c.hi2; c.hi2 = hi[c.q + 2];
    }
    const int s = (int)(bit & 63);
    wlo = funnel64(c.lo0, c.lo1, s);
    whi = funnel64(c.hi0, c.hi1, s);
}

// Pattern masks of a read window from its planes: bit p of PM[c] is 0 iff
// P[mw-1-p] == c (bits p >= mw are 1).
__device__ __forceinline__ void pm_from_planes(u64 pl, u64 ph, int mw, u64 pm[4]) {
    const int sh = 64 - mw;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const u64 eq = ((c & 1) ? pl : ~pl) & ((c & 2) ? ph : ~ph);
        pm[c] = ~(__builtin_bitreverse64(eq) >> sh);
    }
}


// Writes PMT (PM[T[i]] for the window's columns, ~0 at nw..64) into LDS.
template <int G>
__device__ __forceinline__ void store_pmt(u64* lds, int gl, const u64 pm[4], u64 tl, u64 th, int nw) {
    u64* pmt = lds + OFF_PMT;
#pragma unroll
    for (int u = 0; u < 64 / G; ++u) {
        const int i = gl + u * G;
        const int c = (int)((tl >> i) & 1ull) | ((int)((th >> i) & 1ull) << 1);
        pmt[i] = i < nw ? pick_pm(pm[0], pm[1], pm[2], pm[3], c) : ~0ull;
    }
    if (gl == 0) pmt[64] = ~0ull;
}

// PMT of a G-lane group on the step-ordered layout (see SoLayout): entries
// x = -(G-1)..64.
template <int G>
__device__ __forceinline__ void store_pmt_so(u64* lds, int gl, const u64 pm[4], u64 tl, u64 th, int nw) {
    u64* pmt = lds + SoLayout<G>::pmt;
#pragma unroll
    for (int u = 0; u < (64 + G + G - 1) / G; ++u) {
        const int x = gl - (G - 1) + G * u;
        const int i = nw - 1 - x;  // column
        const int sh = i & 63;
        const int c = (int)((tl >> sh) & 1ull) | ((int)((th >> sh) & 1ull) << 1);
        pmt[x] = (x >= 0 && x < nw) ? pick_pm(pm[0], pm[1], pm[2], pm[3], c) : ~0ull;
    }
}

// ---------------------------------------------------------------------------
// DC: one pass of G rows over a window
// ---------------------------------------------------------------------------

// Computes rows c*G .. c*G+G-1 (this lane: row c*G+gl) over columns nw-1..0.
// Stores columns 0..Lc of the row (slots 1..Lc+1 of its table row; slot 0 and
// Lc+2 absorb the out-of-window steps), including column nw (its initial
// value) when nw <= W-O, so that the traceback never special-cases it. Lane
// G-1 writes its row into the boundary row, which lane 0 of the next pass
// reads as the row above. FIRST: pass 0, whose row above is all ones.
template <int G, bool FIRST>
__device__ void dc_pass(u64* lds, int gl, int c, int nw, int Lc, int stride) {
    static_assert(G == 64, "whole-wavefront groups keep every row in LDS");
    const u64* pmt = lds + OFF_PMT;
    u64* brow = lds + OFF_BROW;
    const int d = c * G + gl;
    u64* trow = lds + OFF_TAB + d * stride;
    u64 R = init_word(d);
    u64 Dp = d == 0 ? ~0ull : init_word(d - 1);
    const u64 lowin = d == 0 ? 1ull : 0ull;
    if (Lc == nw) trow[1 + nw] = R;  // lane 0 of a pass never computes column nw
    const int steps = nw + G - 1;
    constexpr int U = 4;
    u64 qpm[U], qov[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int i = nw - 1 - u + gl;
        qpm[u] = pmt[clampi(i, 0, nw)];
        qov[u] = FIRST ? ~0ull : brow[1 + clampi(i, -1, nw + 1)];
    }
    for (int t0 = 0; t0 < steps; t0 += U) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = nw - 1 - (t0 + u) + gl;
            const u64 pm_t = qpm[u];
            const u64 ov = qov[u];
            // operands of step t0+u+U (its column is i-U); the boundary row entry it
            // reads is written by lane G-1 only G-1+U steps later
            const int ip = i - U;
            qpm[u] = pmt[clampi(ip, 0, nw)];
            if (!FIRST) qov[u] = brow[1 + clampi(ip, -1, nw + 1)];
            const u64 up = shift_up<G>(ov, R, gl);
            R = dc_step(R, Dp, up, pm_t, lowin);
            Dp = up;
            trow[1 + clampi(i, -1, Lc + 1)] = R;
            if (gl == G - 1) brow[1 + clampi(i, -1, nw + 1)] = R;
        }
    }
}

// dc_pass for 16- and 32-lane groups on the step-ordered layout (see
// SoLayout): the same computation, with the operand reads and the
// boundary-row write at per-step constant offsets and one clamp for the table
// store.
//
// SINK: the boundary-row store is made by every lane, lane g writing BROW[t-g]
// at step t: lane G-1 its own entry, the others an entry that lane 0 of this
// pass has already read and that lane G-1 writes again later (or, for the
// columns up to Lc, fill_brow before a next pass), so that the store needs no
// execution mask and a group's G words are adjacent. Every such entry lies at
// or below BROW[63] (t - g < nw + G - 2 - Lc, and nw - Lc <= 66 - G when
// L >= G - 2, which the caller checks) and at or above BROW[-(G-1)].
template <int G, bool SPILL, bool FIRST, int U = 8, bool SINK = false>
__device__ void dc_pass_so(u64* lds, u64* spill, int gl, int c, int nw, int Lc, int stride,
                           int lds_rows) {
    using Lay = SoLayout<G>;
    const int d = c * G + gl;
    u64* trow = lds + Lay::tab + d * stride;
    // spilled pass: this lane's column of the pass's step-ordered block (slot t+1
    // holds the entry of step t, slot 0 column nw)
    u64* sp = SPILL ? spill + (size_t)((d - lds_rows) / G) * spill_pass_words(G) + gl : nullptr;
    const u64* pp = lds + Lay::pmt - gl;   // + t: PMT[t - gl]
    const u64* bp = lds + Lay::brow;       // + t: BROW[t]
    u64* bw = lds + Lay::brow - (G - 1);   // + t: BROW[t - (G-1)]
    u64* bsink = bw + (G - 1 - gl);  // + t: BROW[t - gl]
    u64 R = init_word(d);
    u64 Dp = d == 0 ? ~0ull : init_word(d - 1);
    const u64 lowin = d == 0 ? 1ull : 0ull;
    if (Lc == nw) {  // lane 0 of a pass never computes column nw
        if constexpr (SPILL) sp[gl * G] = R;
        else trow[1 + nw] = R;
    }
    const int slot0 = nw + gl;       // table slot 1 + i at t = 0 (column i = nw - 1 - t + gl)
    const int hi_slot = Lc + 2;
    const int steps = nw + G - 1;
    u64 qpm[U], qov[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        qpm[u] = pp[u];
        qov[u] = FIRST ? ~0ull : bp[u];
    }
    // U steps from t0; the table store is left out while every lane's column is
    // above Lc + 1 (those stores go to the dummy slot)
    auto chunk = [&](int t0, auto store, auto brow_store) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int t = t0 + u;
            const u64 pm_t = qpm[u];
            const u64 ov = qov[u];
            const u64 up = shift_up<G>(ov, R, gl);
            R = dc_step(R, Dp, up, pm_t, lowin);
            Dp = up;
            if constexpr (decltype(store)::value) {
                if constexpr (SPILL) sp[(t + 1) * G] = R;
                else trow[med3i(slot0 - t, 0, hi_slot)] = R;
            }
            if constexpr (decltype(brow_store)::value) {
                if constexpr (SINK) bsink[t] = R;
                else if (gl == G - 1) bw[t] = R;
            }
            // operands of steps t+U-1 and t+U, loaded in pairs of adjacent words
            // after both slots' last use (no register copies); the boundary
            // entries were written by lane G-1 at those steps of the previous
            // pass, and this pass's lane G-1 writes entry t+U only at step t+U+G-1
            if (u & 1) {
                qpm[u - 1] = pp[t - 1 + U];
                qpm[u] = pp[t + U];
                if (!FIRST) {
                    qov[u - 1] = bp[t - 1 + U];
                    qov[u] = bp[t + U];
                }
            }
        }
    };
    // lane g stores into slot min(nw + g - t, Lc + 2): the dummy for every lane
    // while t <= nw - Lc - 2. Lane G-1's boundary-row entries for columns <= Lc
    // (steps t >= nw + G - 2 - Lc) are left out: the table row holds them, and
    // fill_brow copies them when a next pass needs the boundary row.
    using yes = std::integral_constant<bool, true>;
    using no = std::integral_constant<bool, false>;
    const int t_free = nw - Lc - 1;
    const int t_bskip = nw + G - 2 - Lc;
    int t0 = 0;
    for (; t0 + U <= t_free; t0 += U) chunk(t0, no{}, yes{});
    for (; t0 < steps && t0 < t_bskip; t0 += U) chunk(t0, yes{}, yes{});
    for (; t0 < steps; t0 += U) chunk(t0, yes{}, no{});
}

// Completes the boundary row entering pass c >= 1 (the last row of pass c-1):
// its entries for columns 0..Lc come from that row's table slots (LDS, or the
// spill for rows at or above lds_rows).
template <int G>
__device__ __forceinline__ void fill_brow(u64* lds, const u64* spill, int gl, int c, int nw, int Lc,
                                          int stride, int lds_rows) {
    const int r = c * G - 1;
    const u64* row = lds + SoLayout<G>::tab + r * stride;
    u64* b = lds + SoLayout<G>::brow;
    for (int col = gl; col <= Lc && col < nw; col += G) {
        const u64 v = r >= lds_rows ? load_spill(spill_entry<G>(spill, r, col, nw, lds_rows))
                                    : row[1 + col];
        b[nw - 1 - col] = v;
    }
}

// ---------------------------------------------------------------------------
// Start search: rows 0.. of the first read window against the whole reference
// ---------------------------------------------------------------------------

// keep ? hit : t, bitwise (keep is all ones or zero), in one v_bfi_b32.
__device__ __forceinline__ int keep_or(int keep, int hit, int t) {
#if defined(__HIP_DEVICE_COMPILE__)
    int r;
    asm("v_bfi_b32 %0, %1, %2, %3" : "=v"(r) : "v"(keep), "v"(hit), "s"(t));
    return r;
#else
    return (keep & hit) | (~keep & t);
#endif
}

// RS rows per lane: slot s of lane gl is row s*G + gl, lagging slot s-1 by G
// steps; lane 0 of slot s takes lane G-1 of slot s-1 through the rotation.
// Returns (in *row, *col) the least row <= Kr with a hit and its leftmost
// column, or row = -1 when rows 0..min(Kr, RS*G-1) have none.
//
// Word form. The pattern sits in the top bits: with a = 64 - m1, bit q + a
// stands for bit q of the usual form and bits below a stay 0 (pattern
// positions that match every base: zero masks and initial bits, and the zero
// that a left shift brings in keeps them zero), so the top pattern bit is bit
// 63 for every read. Each word is kept as its even bits E and odd bits O (bit
// 2k in E bit k, bit 2k+1 in O bit k): a left shift by one is then E' = O << 1,
// O' = E, one 32-bit shift instead of a 64-bit one, and bit 63 is the sign of
// O. The recurrence is unchanged bit for bit.
template <int G, int RS>
__device__ void search_rows(u64* lds, int gl, int lane, const uint8_t* refs, uint64_t fb, int n,
                            int m1, int Kr, int* row_out, int* col_out, int out_hi = 0x7fffffff) {
    static_assert(G == 16 || G == 64, "search groups of 16 or 64 lanes");
    constexpr int BPL = 64 / G;  // text bases each lane converts per 64-column block
    constexpr int O = RS * G;
    constexpr int kRot = G == 16 ? kDppRowRor1 : kDppWaveRor1;
    const int a = 64 - m1;
    const u64 p0 = split_even_odd(lds[OFF_PM + 0] << a), p1 = split_even_odd(lds[OFF_PM + 1] << a),
              p2 = split_even_odd(lds[OFF_PM + 2] << a), p3 = split_even_odd(lds[OFF_PM + 3] << a);
    // text masks by column i at ring word (-i) & 127, and again 128 words on:
    // the steps of a block read increasing words
    u64* ring = lds + kSearchRingOff;
    // columns n..n+63 lie past the text end: the all-mismatch mask
    const u64 past = split_even_odd(~0ull << a);
#pragma unroll
    for (int u = 0; u < BPL; ++u) {
        const int w = (-(n + gl * BPL + u)) & 127;
        ring[w] = past;
        ring[w + 128] = past;
    }

    uint32_t RE[RS], RO[RS], DE[RS], DO[RS];
    int hit[RS];  // step of the last hit (leftmost column so far), -1 before any
#pragma unroll
    for (int s = 0; s < RS; ++s) {
        const int d = s * G + gl;
        const u64 r = split_even_odd(init_word(d) << a);
        const u64 dp = d == 0 ? ~0ull : split_even_odd(init_word(d - 1) << a);
        RE[s] = (uint32_t)r;
        RO[s] = (uint32_t)(r >> 32);
        DE[s] = (uint32_t)dp;
        DO[s] = (uint32_t)(dp >> 32);
        hit[s] = -1;
    }
    // lane 0 of slot 0 (row 0) has no row above: all ones, and a one shifted in
    const uint32_t top = gl == 0 ? ~0u : 0u;
    const uint32_t lowin = gl == 0 ? 1u : 0u;

    auto fetch = [&](int blk) -> unsigned {
        const int c0 = n - 64 * (blk + 1) + gl * BPL;
        unsigned v = 0;
#pragma unroll
        for (int u = 0; u < BPL; ++u) {
            const int col = c0 + u;
            if (col >= 0 && col < n) v |= (unsigned)base_at(refs, fb + col) << (2 * u);
        }
        return v;
    };

    const int steps = n + O - 1;
    const int nblk = (steps + 63) / 64;
    unsigned cur = fetch(0);
    // One block of 64 steps. Slot s of lane gl is at column b - tt at step tt
    // of the block (b = n-1-t0+s*G+gl): ring word ((-b) & 127) + tt, one base
    // address per block, constant offsets, two steps per paired read. EDGE:
    // some lane's column lies outside [0, out_hi) at some step, so hits are
    // range-checked.
    auto block = [&](int t0, auto edge) {
        const u64* rp[RS];
#pragma unroll
        for (int s = 0; s < RS; ++s) rp[s] = ring + ((-(n - 1 - t0 + s * G + gl)) & 127);
        uint32_t pmE[RS][2], pmO[RS][2];
#pragma unroll 8
        for (int tt = 0; tt < 64; ++tt) {
            const int t = t0 + tt;
            uint32_t rE[RS], rO[RS];
#pragma unroll
            for (int s = 0; s < RS; ++s) {
                rE[s] = (uint32_t)__builtin_amdgcn_mov_dpp((int)RE[s], kRot, 0xF, 0xF, false);
                rO[s] = (uint32_t)__builtin_amdgcn_mov_dpp((int)RO[s], kRot, 0xF, 0xF, false);
            }
            if ((tt & 1) == 0) {
#pragma unroll
                for (int s = 0; s < RS; ++s) {
                    const u64 c0 = rp[s][tt], c1 = rp[s][tt + 1];
                    pmE[s][0] = (uint32_t)c0;
                    pmO[s][0] = (uint32_t)(c0 >> 32);
                    pmE[s][1] = (uint32_t)c1;
                    pmO[s][1] = (uint32_t)(c1 >> 32);
                }
            }
#pragma unroll
            for (int s = 0; s < RS; ++s) {
                // the row above at this column: the rotation, with lane 0 taking
                // all ones (slot 0) or lane G-1 of the slot before
                uint32_t uE, uO;
                if (s == 0) {
                    uE = rE[0] | top;
                    uO = rO[0] | top;
                } else {
                    uE = (top & rE[s - 1]) | (~top & rE[s]);
                    uO = (top & rO[s - 1]) | (~top & rO[s]);
                }
                // x = D & (((D & up) << 1) | low); R = x & ((R << 1) | PM)
                const uint32_t eE = DE[s] & uE, eO = DO[s] & uO;
                const uint32_t xE = DE[s] & ((eO << 1) | (s == 0 ? lowin : 0u)), xO = DO[s] & eE;
                const uint32_t sE = (RO[s] << 1) | pmE[s][tt & 1], sO = RE[s] | pmO[s][tt & 1];
                RE[s] = xE & sE;
                RO[s] = xO & sO;
                DE[s] = uE;
                DO[s] = uO;
                if constexpr (decltype(edge)::value) {
                    const int i = n - 1 - t + s * G + gl;
                    const bool h = (int)RO[s] >= 0 && i >= 0 && i < out_hi;
                    hit[s] = h ? t : hit[s];
                } else {
                    hit[s] = keep_or((int)RO[s] >> 31, hit[s], t);  // all ones: no hit
                }
            }
        }
    };
    // block b covers steps 64b..64b+63; lane gl of slot s is at column
    // n-1-t+s*G+gl, so the block is interior when 64b+63 <= n-1 (every column
    // >= 0) and n-1-64b+RS*G-1 < out_hi
    for (int blk = 0; blk < nblk; ++blk) {
        // fill ring entries of this block's columns, prefetch the next block's bases
        const int c0 = n - 64 * (blk + 1) + gl * BPL;
#pragma unroll
        for (int u = 0; u < BPL; ++u) {
            const int w = (-(c0 + u)) & 127;
            const u64 v = pick_pm(p0, p1, p2, p3, (cur >> (2 * u)) & 3);
            ring[w] = v;
            ring[w + 128] = v;
        }
        cur = fetch(blk + 1);
        wave_sync();
        const int t0 = blk * 64;
        const bool interior = t0 + 63 <= n - 1 && n - 1 - t0 + O - 1 < out_hi;
        if (interior) block(t0, std::integral_constant<bool, false>{});
        else block(t0, std::integral_constant<bool, true>{});
        wave_sync();
    }
    // steps of the hits to their columns
#pragma unroll
    for (int s = 0; s < RS; ++s) hit[s] = hit[s] >= 0 ? n - 1 - hit[s] + s * G + gl : -1;
    // least row with a hit
    int row = -1;
#pragma unroll
    for (int s = RS - 1; s >= 0; --s) {
        const int d = s * G + gl;
        const u64 bits = group_ballot(hit[s] >= 0 && d <= Kr, G, lane);
        if (bits) {
            const int w = __builtin_ctzll(bits);
            row = s * G + w;
            if (gl == w) lds[OFF_BC] = (u64)(unsigned)hit[s];
        }
    }
    wave_sync();
    *row_out = row;
    *col_out = row >= 0 ? (int)(unsigned)lds[OFF_BC] : 0;
    wave_sync();
}

// ---------------------------------------------------------------------------
// One pair: windows (DC passes + TB + stitching), run by all G lanes of a group
// ---------------------------------------------------------------------------

struct PairCursor {
    uint64_t rb, fb;      // read / reference stream base offsets
    int m, n;
    int ti, pj;
};

struct TbOut {
    int i_end, j_end, edits;
    uint32_t reads;  // table words read
    bool internal;
};

// Run-length CIGAR under construction, kept with the same values in every lane
// of a group. The runs of the current window go to an LDS array (`runs`, the
// boundary-row area, free during the traceback), written with the same value
// by every lane of the group: slot nr holds the open run and is rewritten at
// every step, and nr moves on when the op changes, so a step needs no branch. At the end of each window the group
// copies the closed runs to device memory; the open run is carried into the
// next window's slot 0, so runs merge across window seams.
struct RunState {
    int cur_op;         // op of the open run, -1 before the pair's first op
    uint32_t cur_len;
    int nr;             // LDS slot of the open run, -1 before the pair's first op
};

__device__ __forceinline__ void run_push(uint32_t* runs, RunState& rs, int op, uint32_t count,
                                         bool writer) {
    const bool changed = op != rs.cur_op;
    rs.nr += changed ? 1 : 0;
    rs.cur_len = changed ? count : rs.cur_len + count;
    rs.cur_op = op;
    // every lane of the group stores the same word to the same slot: no
    // execution mask to set up around the store
    (void)writer;
    runs[rs.nr] = (rs.cur_len << 2) | (uint32_t)op;
}

// Before a window's traceback: the open run moves to slot 0.
__device__ __forceinline__ void run_window_start(uint32_t* runs, RunState& rs, bool writer) {
    if (rs.nr >= 0) {
        if (writer) runs[0] = (rs.cur_len << 2) | (uint32_t)rs.cur_op;
        rs.nr = 0;
    }
}

__device__ __forceinline__ int ctz64(u64 x) { return x ? __builtin_ctzll(x) : 64; }

// Traceback of one window from (i=0, j=0, d=dstar) (j = read bases consumed,
// bit p = mw-1-j), run by every lane of the group on the same values; `writer`
// marks the one lane that writes run records.
//
// Edge order M, S, I, D. The current cell is valid at every step (bit p of
// R[d][i] is 0), and then the match edge is valid exactly when i < nw and the
// two bases are equal: R[d][i] bit p = 0 says the read suffix from j aligns to
// a prefix of the text suffix from i within d edits, and when the first bases
// agree the suffixes after them align within the same d edits (the usual
// equal-first-character property of edit distance, which also holds with a free
// text end). So a run of matches is the common prefix of the read and text
// from (j, i), found from the bit planes with one XOR and a trailing-zero
// count, and only the other three edges read the table: substitution and
// deletion test R[d-1][i+1] (bit p-1 and bit p), insertion tests R[d-1][i]
// (bit p-1), with "p == 0 or bit p-1 is 0" taken as bit p of the word
// shifted left by one.
//
// Rows at or above lds_rows come from the group's spill in device memory. Each
// edit there also loads, one word per lane of the group, columns i..i+G-1 of
// the row below (the row the next edit reads, since every edit lowers d by
// one); when the next edit's two columns fall inside that range it takes them
// from the loading lanes instead of from memory, so a spilled edit waits for
// one load issued an edit earlier rather than for its own.
template <int G>
__device__ __forceinline__ TbOut traceback_planes(const u64* lds, const u64* spill, uint32_t* runs, RunState& rs,
                                  bool writer, u64 pl, u64 ph, u64 tl, u64 th, int mw, int nw,
                                  int dstar, int L, int stride, int lds_rows, int gl, int lane,
                                  bool prefetch) {
    const u64* tab = lds + tab_off<G>() + 1;  // column c of a row sits in slot c + 1
    const int jmax = min(mw, L);
    int i = 0, j = 0, d = dstar;
    TbOut o{0, 0, 0, 0u, false};
    u64 pf = 0;            // this lane's word of the prefetched row
    int pf_row = -1, pf_col = 0;
    const int gbase = lane - gl;
    // word offset of row d-1 (every edit lowers d by one: no multiply per edit)
    int roff = (dstar - 1) * stride;
    // every pass of the loop consumes a read or text base, or leaves it
    for (int it = 0; it <= 2 * L; ++it) {
        if (j >= jmax || i >= L) break;
        // read bases j.. against text bases i.. (j, i < 64 here; the zeros shifted
        // in past the words are cut by the limits below)
        const u64 mis = ((pl >> j) ^ (tl >> i)) | ((ph >> j) ^ (th >> i));
        const int k = min(ctz64(mis), min(jmax - j, min(L - i, nw - i)));
        {
            // the match run, without a branch: with k = 0 nothing changes and the
            // open run's record is rewritten (slot 0 before the pair's first op,
            // which that op then overwrites)
            const bool push = k > 0;
            const bool changed = push && rs.cur_op != (int)GENASM_OP_MATCH;
            rs.nr += changed ? 1 : 0;
            rs.cur_len = changed ? (uint32_t)k : rs.cur_len + (uint32_t)k;
            rs.cur_op = push ? (int)GENASM_OP_MATCH : rs.cur_op;
            runs[max(rs.nr, 0)] = (rs.cur_len << 2) | (uint32_t)rs.cur_op;
            i += k;
            j += k;
            if (j >= jmax || i >= L) break;
        }
        // bases differ, or the text window is used up: an edit
        if (d < 1) { o.internal = true; break; }
        const int r = d - 1, p = mw - 1 - j;
        u64 B, C;
        if (r < lds_rows) {
            const u64* row = tab + roff;
            C = row[i];
            B = row[i + 1];
        } else {
            const bool hit = r == pf_row && i >= pf_col && i + 1 < pf_col + G;
            const int src = gbase + (i - pf_col);
            const u64 have = pf;
            // the row below, for the next edit, before this edit waits for its words
            if (prefetch && r - 1 >= lds_rows) {
                pf = load_spill(spill_entry<G>(spill, r - 1, min(i + gl, L), nw, lds_rows));
                pf_row = r - 1;
                pf_col = i;
            } else {
                pf_row = -1;
            }
            if (hit) {
                C = __shfl(have, src);
                B = __shfl(have, src + 1);
            } else {
                C = load_spill(spill_entry<G>(spill, r, i, nw, lds_rows));
                B = load_spill(spill_entry<G>(spill, r, i + 1, nw, lds_rows));
            }
        }
        const bool intext = i < nw;
        const bool s_ok = intext && !(((B << 1) >> p) & 1ull);
        const bool i_ok = !(((C << 1) >> p) & 1ull);
        const bool d_ok = intext && !((B >> p) & 1ull);
        if (!(s_ok || i_ok || d_ok)) { o.internal = true; break; }
        const int op = s_ok ? GENASM_OP_MISMATCH : i_ok ? GENASM_OP_INS : GENASM_OP_DEL;
        run_push(runs, rs, op, 1u, writer);
        o.reads += 2u;
        i += op != GENASM_OP_INS;
        j += op != GENASM_OP_DEL;
        d -= 1;
        roff -= stride;
    }
    o.i_end = i;
    o.j_end = j;
    o.edits = dstar - d;
    return o;
}

// Copies runs [0, count) of the group's LDS run array to the pair's CIGAR in
// device memory at element `written`; all lanes of the group take part.
template <int G>
__device__ __forceinline__ bool copy_runs(const uint32_t* runs, int count, uint32_t* cigar,
                                          uint64_t base, uint64_t limit, uint32_t written, int gl) {
    bool overflow = false;
    for (int k = gl; k < count; k += G) {
        const uint64_t idx = base + written + (uint64_t)k;
        if (idx < limit) cigar[idx] = runs[k];
        else overflow = true;
    }
    return overflow;
}

__device__ __forceinline__ PairCursor pair_cursor(const AlignParams& P, uint64_t pair) {
    PairCursor pc;
    pc.rb = P.read_off[pair];
    pc.fb = P.ref_off[pair];
    pc.m = (int)(P.read_len ? P.read_len[pair] : P.read_off[pair + 1] - pc.rb);
    pc.n = (int)(P.ref_len ? P.ref_len[pair] : P.ref_off[pair + 1] - pc.fb);
    pc.ti = pc.pj = 0;
    return pc;
}

__device__ __forceinline__ uint64_t pair_run_base(const AlignParams& P, uint64_t pair) {
    return P.run_base ? P.run_base[pair]
                      : (P.read_off[pair] - P.read_off[0]) + (P.ref_off[pair] - P.ref_off[0]);
}

__device__ __forceinline__ PairState fresh_state(int s) {
    return PairState{s, 0, 0, 0u, 0u, -1, 0u, kStateStarted};
}

// A resident pair's turn in a serving iteration (inactive elsewhere). The
// device clock is read by a scalar instruction and the two counters are made
// wave-uniform, so every lane of a group takes the same branch. The counters
// are looked at no more often than every kTurnLookTicks per group: the
// arrival count is written by a host-to-device copy while the kernel runs, so
// it is read past the caches.
constexpr u64 kTurnLookTicks = 2000;  // 20 us
struct TurnClock {
    u64 end = 0, soon = 0, admitted = 0, next_look = 0;
    const unsigned long long* arrivals = nullptr;
    const uint32_t* fin_len = nullptr;
    bool active = false;
    __device__ __forceinline__ void open(const AlignParams& P) {
        if (!P.turn) return;
        const TurnLimits t = *P.turn;
        end = t.end;
        soon = t.soon;
        admitted = t.admitted;
        arrivals = P.arrivals;
        fin_len = P.fin_len;
        active = true;
    }
    // Whether the turn has ended (asked before every window but the first).
    __device__ __forceinline__ bool over() {
        const u64 now = wall_clock64();
        if (now >= end) return true;
        if (now < soon || now < next_look) return false;
        next_look = now + kTurnLookTicks;
        const u64 a = arrivals ? __hip_atomic_load(arrivals, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM) : 0ull;
        const uint32_t f = fin_len ? __hip_atomic_load(fin_len, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0u;
        return __builtin_amdgcn_readfirstlane((int)(a > admitted || f > 0u)) != 0;
    }
};

// Debug builds (GENASM_DEBUG): an invariant guarding the accesses that
// follow; when it fails, the pair's audit word records `bit` (all lanes of the
// group write the same bit) and the caller ends the pair. Release builds
// compile the check away.
__device__ __forceinline__ bool audit_ok(const AlignParams& P, uint64_t pair, uint32_t bit, bool ok) {
#if defined(GENASM_DEBUG)
    if (!ok && P.audit) atomicOr(P.audit + pair, bit);
    return ok;
#else
    (void)P; (void)pair; (void)bit; (void)ok;
    return true;
#endif
}

// Rows of the spill area one G-lane group may use: whole spilled passes of
// its step-ordered blocks in its area (a 32-lane group owning the areas of
// two 16-lane groups); 64-lane groups keep every row in LDS.
template <int G>
__device__ __forceinline__ int spill_capacity(const AlignParams& P) {
    if constexpr (G == 64) return 0;
    else return (G / 16) * spill_group_words(64 - P.lds_rows) / spill_pass_words(G) * G;
}

// Advances one pair whose window state is `st` by at most `budget` windows
// (0: to the end). All G lanes of the group call this together; lane 0 holds
// the traceback-side fields (score, open run). When the pair ends (read
// consumed, or a window without a solution within K) the result and the last
// CIGAR run are written and st gets kStateDone.
template <int G>
__device__ __forceinline__ uint32_t advance_pair(const AlignParams& P, u64* lds, u64* spill, int lds_rows, int gl,
                             int lane, uint64_t pair, const PairCursor& pc, int s, PairState& st,
                             uint32_t budget, TurnClock& turn) {
    const uint64_t run_base = pair_run_base(P, pair);
    const uint64_t run_limit = min(P.cigar_cap, run_base + (uint64_t)pc.m + (uint64_t)pc.n);
    uint32_t* runs = reinterpret_cast<uint32_t*>(lds + runs_off<G>());
    RunState rs{st.cur_op, st.cur_len, st.cur_op >= 0 ? 0 : -1};
    bool overflow = (st.flags & kStateOverflow) != 0;
    bool failed = false, internal = false;
    u64 st_wops = 0, st_cells = 0, st_table = 0, st_tb = 0, st_steps = 0;
    // phase clocks, read only when profiling
    const bool timing = P.stats != nullptr;
    u64 cyc_dc = 0, cyc_tb = 0;
    const u64 cyc_start = timing ? clock64() : 0;
    const u64 wall_start = timing ? wall_clock64() : 0;
    // Every window commits at least one base, so a pair has at most m + n
    // windows; the cap keeps the loop finite even if that ever failed.
    const uint32_t max_windows = (uint32_t)pc.m + (uint32_t)pc.n + 1u;
    uint32_t done_here = 0;
    const bool writer = gl == 0;
    const uint64_t rorg = P.planes_from_off0 ? (P.read_off[0] & ~63ull) : 0;
    const uint64_t forg = P.planes_from_off0 ? (P.ref_off[0] & ~63ull) : 0;
    SeqCursor rc, fc;
    if (st.pj < pc.m) {
        seq_open(rc, P.read_lo, P.read_hi, pc.rb - rorg + st.pj);
        seq_open(fc, P.ref_lo, P.ref_hi, pc.fb - forg + st.ti);
    }
    while (st.pj < pc.m && (budget == 0 || done_here < budget)) {
        // every pair advances at least one window per launch (so that a late
        // start never leaves a pair without progress); no further window
        // starts once its turn has ended
        if (turn.active && done_here > 0 && turn.over()) break;
        if (st.nwin >= max_windows) { failed = true; internal = true; break; }
        const int mw = min(P.W, pc.m - st.pj);
        const int nw = min(P.W, pc.n - st.ti);
        const int Lc = min(nw, P.L);
        if (!audit_ok(P, pair, kAuditWindow,
                      P.W >= 2 && P.W <= 64 && mw >= 1 && nw >= 0 && Lc + 2 <= P.stride)) {
            failed = true;
            internal = true;
            break;
        }
        ++st.nwin;
        ++done_here;
        const u64 cyc0 = timing ? clock64() : 0;
        u64 pl, ph, tl, th;
        seq_window(rc, P.read_lo, P.read_hi, pc.rb - rorg + st.pj, pl, ph);
        seq_window(fc, P.ref_lo, P.ref_hi, pc.fb - forg + st.ti, tl, th);
        // rows that need computing; row mw always solves. With an empty text
        // window every column is the initial one and row mw is the first hit.
        const int Kr = nw > 0 ? min(P.K, mw - 1) : -1;
        if (Kr >= 0) {
            u64 pm[4];
            pm_from_planes(pl, ph, mw, pm);
            if constexpr (G == 64) store_pmt<G>(lds, gl, pm, tl, th, nw);
            else store_pmt_so<G>(lds, gl, pm, tl, th, nw);
            wave_sync();
        }
        int dstar = -1;
        st_cells += (u64)mw * nw;
        bool pass_ok = true;
        const bool sink = P.L >= G - 2;  // the boundary-row store of every lane fits
        for (int c = 0; c * G <= Kr; ++c) {
            st_steps += (u64)G * (nw + G - 1);
            const bool spill_pass = c * G >= lds_rows;
            pass_ok = spill_pass
                ? audit_ok(P, pair, kAuditSpill, (c + 1) * G - lds_rows <= spill_capacity<G>(P))
                : audit_ok(P, pair, kAuditLds, (c + 1) * G <= lds_rows);
            if (!pass_ok) break;
            if constexpr (G != 64) {
                if (c >= 1) {
                    fill_brow<G>(lds, spill, gl, c, nw, Lc, P.stride, lds_rows);
                    wave_sync();
                }
                if (spill_pass) {
                    if (sink) dc_pass_so<G, true, false, 8, true>(lds, spill, gl, c, nw, Lc, P.stride, lds_rows);
                    else dc_pass_so<G, true, false>(lds, spill, gl, c, nw, Lc, P.stride, lds_rows);
                    mem_sync();
                } else {
                    if (c == 0) {
                        if (sink) dc_pass_so<G, false, true, 8, true>(lds, spill, gl, c, nw, Lc, P.stride, lds_rows);
                        else dc_pass_so<G, false, true>(lds, spill, gl, c, nw, Lc, P.stride, lds_rows);
                    } else {
                        if (sink) dc_pass_so<G, false, false, 8, true>(lds, spill, gl, c, nw, Lc, P.stride, lds_rows);
                        else dc_pass_so<G, false, false>(lds, spill, gl, c, nw, Lc, P.stride, lds_rows);
                    }
                    wave_sync();
                }
            } else {
                // 64 rows in LDS: one pass, never spilled (lds_rows is 64)
                dc_pass<G, true>(lds, gl, c, nw, Lc, P.stride);
                wave_sync();
            }
            const int d = c * G + gl;
            const u64 r0 = spill_pass ? load_spill(spill_entry<G>(spill, d, 0, nw, lds_rows))
                                      : lds[tab_off<G>() + d * P.stride + 1];
            const bool sol = d <= Kr && !((r0 >> (mw - 1)) & 1ull);
            const u64 bits = group_ballot(sol, G, lane);
            if (bits) { dstar = c * G + __builtin_ctzll(bits); break; }
        }
        if (!pass_ok) { failed = true; internal = true; break; }
        if (dstar < 0) {
            if (mw <= P.K) dstar = mw;  // no row below mw solves: d* = mw
            else { failed = true; break; }
        }
        const u64 cyc1 = timing ? clock64() : 0;
        // traceback, in every lane of the group on the same values
        TbOut t;
        run_window_start(runs, rs, writer);
        if (nw == 0) {
            // empty text window: every step of the traceback is an insertion
            const int k = min(mw, P.L);
            run_push(runs, rs, GENASM_OP_INS, (uint32_t)k, writer);
            t = TbOut{0, k, k, 0u, false};
        } else {
            t = traceback_planes<G>(lds, spill, runs, rs, writer, pl, ph, tl, th, mw, nw, dstar, P.L,
                                    P.stride, lds_rows, gl, lane, P.tb_prefetch != 0);
        }
        st.score += t.edits;
        st_tb += t.reads;
        st_wops += (u64)nw * (2 + 6 * dstar);
        st_table += (u64)(dstar + 1) * (Lc + 1);
        if (t.internal) { failed = true; internal = true; break; }
        if (!audit_ok(P, pair, kAuditRuns, rs.nr <= 2 * min(P.L, dstar) + 1)) {
            failed = true;
            internal = true;
            break;
        }
        wave_sync();  // run records written by the writer lane
        // closed runs of this window (slots below the open run) go to device memory
        const int closed = max(rs.nr, 0);
        overflow |= copy_runs<G>(runs, closed, P.cigar, run_base, run_limit, st.written, gl);
        st.written += (uint32_t)closed;
        wave_sync();  // the next window's traceback rewrites the run slots
        st.ti += t.i_end;
        st.pj += t.j_end;
        if (timing) {
            const u64 cyc2 = clock64();
            cyc_dc += cyc1 - cyc0;
            cyc_tb += cyc2 - cyc1;
        }
    }
    st.cur_op = rs.cur_op;
    st.cur_len = rs.cur_len;
    const bool finished = failed || st.pj >= pc.m;
    // the open run closes with the pair
    if (finished && !failed && writer && rs.cur_op >= 0) {
        const uint64_t idx = run_base + st.written;
        if (idx < run_limit) P.cigar[idx] = (rs.cur_len << 2) | (uint32_t)rs.cur_op;
        else overflow = true;
    }
    if (group_ballot(overflow, G, lane) != 0) st.flags |= kStateOverflow;
    if (failed) st.flags |= kStateFailed;
    if (internal) st.flags |= kStateInternal;
    if (finished) st.flags |= kStateDone;
    if (gl == 0 && finished) {
        const bool ovf = (st.flags & kStateOverflow) != 0;
        genasm_result r;
        if (failed) {
            r.edit_distance = -1;
            r.ref_begin = r.ref_end = 0;
            r.cigar_len = 0;
        } else {
            r.edit_distance = st.score;
            r.ref_begin = (uint32_t)s;
            r.ref_end = (uint32_t)st.ti;
            r.cigar_len = ovf ? 0u : st.written + (rs.cur_op >= 0 ? 1u : 0u);
        }
        r.n_windows = st.nwin;
        r.cigar_off = run_base;
        r.flags = (ovf && !failed ? GENASM_FLAG_CIGAR_OVERFLOW : 0u) |
                  (internal ? GENASM_FLAG_INTERNAL : 0u);
        P.out[pair] = r;
    }
    if (gl == 0 && P.stats) {
        u64* stp = P.stats + pair * kStatCount;
        stp[kStatWindowWordOps] += st_wops;
        stp[kStatWindowCells] += st_cells;
        stp[kStatTableWords] += st_table;
        stp[kStatTbReads] += st_tb;
        stp[kStatWindowLaneSteps] += st_steps;
        stp[kStatWindows] += done_here;
        stp[kStatDcCycles] += cyc_dc;
        stp[kStatTbCycles] += cyc_tb;
        stp[kStatPairCycles] += clock64() - cyc_start;
        if (!stp[kStatPairStart]) stp[kStatPairStart] = wall_start;
        stp[kStatPairEnd] = wall_clock64();
    }
    return done_here;
}

// Runs (or resumes, when window state persists in P.state) the windows of a
// pair whose start search hit at column s.
template <int G>
__device__ __forceinline__ void run_pair(const AlignParams& P, u64* lds, u64* spill, int lds_rows, int gl,
                         int lane, uint64_t pair, int s) {
#if defined(GENASM_DEBUG)
    if (P.audit && gl == 0) atomicAdd(P.audit + pair, kAuditTake);  // queue audit
#endif
    const PairCursor pc = pair_cursor(P, pair);
    if (!P.state) {
        PairState st = fresh_state(s);
        TurnClock none;
        advance_pair<G>(P, lds, spill, lds_rows, gl, lane, pair, pc, s, st, 0u, none);
        return;
    }
    PairState st = P.state[pair];
    if (st.flags & kStateDone) return;
    if (!(st.flags & kStateStarted)) st = fresh_state(s);
    TurnClock turn;
    turn.open(P);
    const uint32_t advanced =
        advance_pair<G>(P, lds, spill, lds_rows, gl, lane, pair, pc, s, st, P.window_budget, turn);
    if (gl == 0) {
        P.state[pair] = st;
        // serving: the pair's list for the next iteration (hot: its turn was
        // cut after one window, so it goes first next time), or the finished list
        if (P.fin_list) {
            if (st.flags & kStateDone)
                P.fin_list[atomicAdd(P.fin_len, 1u)] = (uint32_t)pair;
            else if (advanced <= 1)
                P.next_hot[atomicAdd(P.next_len + kCounterEasyLen, 1u)] = (uint32_t)pair;
            else
                P.next_cold[atomicAdd(P.next_len + kCounterHardLen, 1u)] = (uint32_t)pair;
        }
    }
}

// Start-search counters of one pair (lane 0); `row` is the hit row or, when
// no row hit, the last row computed. Lane-steps add up over search stages.
__device__ __forceinline__ void search_stats(const AlignParams& P, uint64_t pair, int n, int m1,
                                             int row, u64 lane_steps, bool first_stage) {
    if (!P.stats) return;
    u64* st = P.stats + pair * kStatCount;
    st[kStatSearchWordOps] = (u64)n * (2 + 6 * (u64)max(row, 0));
    st[kStatSearchCells] = (u64)m1 * n;
    st[kStatSearchLaneSteps] = (first_stage ? 0ull : st[kStatSearchLaneSteps]) + lane_steps;
}

// Result of a pair that ends before any window: an empty read (score 0) or a
// start search without a hit within K (score -1).
__device__ __forceinline__ void finish_without_windows(const AlignParams& P, uint64_t pair,
                                                       int32_t score) {
    genasm_result r;
    r.edit_distance = score;
    r.ref_begin = r.ref_end = 0;
    r.n_windows = 0;
    r.cigar_off = pair_run_base(P, pair);
    r.cigar_len = 0;
    r.flags = 0;
    P.out[pair] = r;
    if (P.state) {
        PairState st = fresh_state(0);
        st.flags |= kStateDone | (score < 0 ? kStateFailed : 0u);
        P.state[pair] = st;
    }
}

// ---------------------------------------------------------------------------
// Plain form: one pair per workgroup, 64 lanes = 64 rows
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(64) void k_plain(AlignParams P) {
    extern __shared__ u64 smem[];
    const int lane = threadIdx.x;
    const uint64_t pair = blockIdx.x;
    if (pair >= P.n_pairs) return;
    const PairCursor pc = pair_cursor(P, pair);
    if (pc.m == 0) {
        if (lane == 0) finish_without_windows(P, pair, 0);
        return;
    }
    const int m1 = min(P.W, pc.m);
    const int Kr = min(P.K, m1 - 1);
    build_pm<64>(smem, lane, P.reads, pc.rb, m1, false);
    int row, col;
    search_rows<64, 1>(smem, lane, lane, P.refs, pc.fb, pc.n, m1, Kr, &row, &col);
    if (lane == 0)
        search_stats(P, pair, pc.n, m1, row >= 0 ? row : (m1 <= P.K ? m1 : Kr), 64ull * (pc.n + 63), true);
    if (row < 0) {
        if (m1 <= P.K) { row = m1; col = 0; }   // row m1 hits in every column
        else {
            if (lane == 0) finish_without_windows(P, pair, -1);
            return;
        }
    }
    run_pair<64>(P, smem, nullptr, 64, lane, lane, pair, col);
}

// ---------------------------------------------------------------------------
// Pre-alignment filter (score-only mode)
// ---------------------------------------------------------------------------
//
// The DC recurrence over the whole read (an NW-word bit vector per row, bit p
// = read base m-1-p) against the whole reference, with no table and no
// traceback: the least row d <= k with a column whose top bit is clear is the
// least edit distance between the read and any substring of the reference,
// and the leftmost such column is where that substring starts. One pair per
// 64-lane workgroup; lane d computes row d over an anti-diagonal wavefront of
// the reference columns, as the start search does for one read window.

__device__ __forceinline__ u64 init_word_at(int d, int w) {
    // word w of the initial column of row d: bits below d are 0
    const int lo = 64 * w;
    return d >= lo + 64 ? 0ull : d <= lo ? ~0ull : (~0ull << (d - lo));
}

template <int NW>
__global__ __launch_bounds__(64) void k_filter(const uint8_t* reads, const uint64_t* read_off,
                                               const uint8_t* refs, const uint64_t* ref_off,
                                               uint64_t n_pairs, int32_t K, int32_t* dist,
                                               uint32_t* start) {
    extern __shared__ u64 smem[];
    u64* pm = smem;                                           // 4 x NW words (match masks first)
    uint8_t* ring = reinterpret_cast<uint8_t*>(smem + 4 * NW);  // 128 text codes
    u64* bc = smem + 4 * NW + 16;                             // broadcast slot
    const int lane = threadIdx.x;
    const uint64_t pair = blockIdx.x;
    if (pair >= n_pairs) return;
    const uint64_t rb = read_off[pair], fb = ref_off[pair];
    const int m = (int)(read_off[pair + 1] - rb);
    const int n = (int)(ref_off[pair + 1] - fb);
    if (m == 0) {
        if (lane == 0) { dist[pair] = 0; start[pair] = 0u; }
        return;
    }
    // match masks: bit q of eq[c] is 1 iff read base m-1-q is c; PM[c] = ~eq[c]
    for (int w = lane; w < 4 * NW; w += 64) pm[w] = 0ull;
    wave_sync();
    for (int b = lane; b < m; b += 64) {
        const int q = m - 1 - b;
        atomicOr(&pm[base_at(reads, rb + b) * NW + q / 64], 1ull << (q % 64));
    }
    wave_sync();
    for (int w = lane; w < 4 * NW; w += 64) pm[w] = ~pm[w];
    wave_sync();

    const int d = lane;
    u64 R[NW], Dp[NW];
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        R[w] = init_word_at(d, w);
        Dp[w] = d == 0 ? ~0ull : init_word_at(d - 1, w);
    }
    const u64 lowin = d == 0 ? 1ull : 0ull;
    const int top_w = (m - 1) / 64, top_b = (m - 1) % 64;
    int hit = -1;
    const int steps = n + 63;
    const int nblk = (steps + 63) / 64;
    for (int blk = 0; blk < nblk; ++blk) {
        // codes of this block's 64 columns into the ring (the previous block's stay)
        const int c = n - 64 * (blk + 1) + lane;
        if (c >= 0 && c < n) ring[c & 127] = (uint8_t)base_at(refs, fb + c);
        wave_sync();
        for (int tt = 0; tt < 64; ++tt) {
            const int t = blk * 64 + tt;
            const int i = n - 1 - t + d;
            const bool in = i >= 0 && i < n;
            const int code = in ? ring[i & 127] : 0;
            u64 up[NW], a[NW];
#pragma unroll
            for (int w = 0; w < NW; ++w) {
                up[w] = LaneShift<64>::up(~0ull, R[w]);
                a[w] = Dp[w] & up[w];
            }
            u64 Rn[NW];
#pragma unroll
            for (int w = 0; w < NW; ++w) {
                const u64 ash = (a[w] << 1) | (w ? (a[w - 1] >> 63) : lowin);
                const u64 rsh = (R[w] << 1) | (w ? (R[w - 1] >> 63) : 0ull);
                const u64 pmw = in ? pm[code * NW + w] : ~0ull;
                Rn[w] = (Dp[w] & ash) & (rsh | pmw);
            }
#pragma unroll
            for (int w = 0; w < NW; ++w) {
                R[w] = Rn[w];
                Dp[w] = up[w];
            }
            if (in && d <= K && !((R[top_w] >> top_b) & 1ull)) hit = i;  // columns fall: leftmost last
        }
        wave_sync();  // the next block overwrites ring entries of the block before last
    }
    // rows at or above m also match the empty substring at column n
    if (hit < 0 && d >= m && d <= K) hit = n;
    const u64 bits = __ballot(hit >= 0 && d <= K);
    if (bits) {
        const int row = __builtin_ctzll(bits);
        if (lane == row) bc[0] = (u64)(unsigned)hit;
        wave_sync();
        if (lane == 0) {
            dist[pair] = row;
            start[pair] = (uint32_t)bc[0];
        }
    } else if (lane == 0) {
        dist[pair] = -1;
        start[pair] = 0u;
    }
}

int filter_words(uint32_t max_read_len) {
    return max_read_len <= 64 ? 1 : max_read_len <= 128 ? 2 : max_read_len <= 256 ? 4
         : max_read_len <= 512 ? 8 : max_read_len <= 1024 ? 16 : 0;
}

hipError_t launch_filter(const uint8_t* reads, const uint64_t* read_off, const uint8_t* refs,
                         const uint64_t* ref_off, uint64_t n_pairs, uint32_t max_read_len,
                         int32_t k, int32_t* dist, uint32_t* start, hipStream_t s) {
    if (n_pairs == 0) return hipSuccess;
    const int NW = filter_words(max_read_len);
    const int K = k < 63 ? k : 63;
    const size_t lds = (4 * (size_t)NW + 16 + 1) * 8;
    const dim3 grid((unsigned)n_pairs), block(64);
    switch (NW) {
        case 1: hipLaunchKernelGGL(k_filter<1>, grid, block, lds, s, reads, read_off, refs, ref_off, n_pairs, K, dist, start); break;
        case 2: hipLaunchKernelGGL(k_filter<2>, grid, block, lds, s, reads, read_off, refs, ref_off, n_pairs, K, dist, start); break;
        case 4: hipLaunchKernelGGL(k_filter<4>, grid, block, lds, s, reads, read_off, refs, ref_off, n_pairs, K, dist, start); break;
        case 8: hipLaunchKernelGGL(k_filter<8>, grid, block, lds, s, reads, read_off, refs, ref_off, n_pairs, K, dist, start); break;
        case 16: hipLaunchKernelGGL(k_filter<16>, grid, block, lds, s, reads, read_off, refs, ref_off, n_pairs, K, dist, start); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Unimproved form (ablation): the GenASM window without the three improvements
// ---------------------------------------------------------------------------
//
// One pair per 64-lane workgroup, as the plain form, but each window computes
// every row 0..K (no early exit), keeps all four edge words (match,
// substitution, insertion, deletion) of every entry (d, i), i < nw (no AND,
// no pruning of unreachable entries) in device memory, reads d* off column 0
// afterwards, and traces back by testing bit p of the stored edge words. Lane
// d computes row d; when K = 64, lane 63 also computes row 64 from its own
// row. Results equal the improved forms (the edges are pure functions of R).

// Edge words of entry (d, i): table + ((d * 64) + i) * 4 + {0 M, 1 S, 2 I, 3 D}.
constexpr int kUnimpRows = 65;
constexpr uint64_t kUnimpWords = (uint64_t)kUnimpRows * 64 * 4;  // per workgroup

__device__ __forceinline__ void store_edges(u64* e, u64 m, u64 s, u64 in, u64 d) {
    e[0] = m;
    e[1] = s;
    e[2] = in;
    e[3] = d;
}

__device__ TbOut traceback_unimproved(const u64* tab, uint32_t* runs, RunState& rs, bool writer,
                                      u64 pl, u64 ph, u64 tl, u64 th, int mw, int nw, int dstar,
                                      int L, bool& internal) {
    int i = 0, p = mw - 1, d = dstar;
    TbOut o{0, 0, 0, 0u, false};
    while (p >= 0 && i < L && mw - 1 - p < L) {
        const int j = mw - 1 - p;
        const bool intext = i < nw;
        u64 m = ~0ull, sw = ~0ull, iw = ~0ull, dw = ~0ull;
        if (intext) {
            const u64* e = tab + ((size_t)d * 64 + i) * 4;
            m = load_spill(e + 0);
            if (d >= 1) {
                sw = load_spill(e + 1);
                iw = load_spill(e + 2);
                dw = load_spill(e + 3);
            }
        } else if (d >= 1) {
            iw = init_word(d - 1) << 1;  // past the text end only the insertion edge exists
        }
        const bool m_ok = !((m >> p) & 1ull);
        const bool s_ok = d >= 1 && !((sw >> p) & 1ull);
        const bool i_ok = d >= 1 && !((iw >> p) & 1ull);
        const bool d_ok = d >= 1 && !((dw >> p) & 1ull);
        // words an edge-by-edge traceback reads: the match word when the bases
        // agree, then each further edge word tested, in priority order
        const bool eq = intext && !((((pl >> j) ^ (tl >> i)) | ((ph >> j) ^ (th >> i))) & 1ull);
        const uint32_t more = (d >= 1 && intext) ? 1u : 0u;
        o.reads += (eq ? 1u : 0u) +
                   (m_ok ? 0u : more * (s_ok ? 1u : i_ok ? 2u : 3u));
        if (!(m_ok || s_ok || i_ok || d_ok)) { internal = true; break; }
        const int op = m_ok ? GENASM_OP_MATCH : s_ok ? GENASM_OP_MISMATCH
                     : i_ok ? GENASM_OP_INS : GENASM_OP_DEL;
        run_push(runs, rs, op, 1u, writer);
        i += op != GENASM_OP_INS;
        p -= op != GENASM_OP_DEL;
        d -= op != GENASM_OP_MATCH;
    }
    o.i_end = i;
    o.j_end = mw - 1 - p;
    o.edits = dstar - d;
    return o;
}

__global__ __launch_bounds__(64) void k_unimproved(AlignParams P, u64* table) {
    extern __shared__ u64 smem[];
    const int lane = threadIdx.x;
    const uint64_t pair = blockIdx.x;
    if (pair >= P.n_pairs) return;
    const PairCursor pc = pair_cursor(P, pair);
    if (pc.m == 0) {
        if (lane == 0) finish_without_windows(P, pair, 0);
        return;
    }
    const int m1 = min(P.W, pc.m);
    const int Kr = min(P.K, m1 - 1);
    build_pm<64>(smem, lane, P.reads, pc.rb, m1, false);
    int row, col;
    search_rows<64, 1>(smem, lane, lane, P.refs, pc.fb, pc.n, m1, Kr, &row, &col);
    if (lane == 0)
        search_stats(P, pair, pc.n, m1, row >= 0 ? row : (m1 <= P.K ? m1 : Kr), 64ull * (pc.n + 63), true);
    if (row < 0) {
        if (m1 <= P.K) { row = m1; col = 0; }
        else {
            if (lane == 0) finish_without_windows(P, pair, -1);
            return;
        }
    }
    u64* tab = table + pair * kUnimpWords;
    const uint64_t run_base = pair_run_base(P, pair);
    const uint64_t run_limit = min(P.cigar_cap, run_base + (uint64_t)pc.m + (uint64_t)pc.n);
    uint32_t* runs = reinterpret_cast<uint32_t*>(smem + OFF_BROW);
    const bool writer = lane == 0;
    RunState rs{-1, 0u, -1};
    int ti = col, pj = 0, score = 0;
    uint32_t nwin = 0, written = 0;
    bool overflow = false, failed = false, internal = false;
    u64 st_wops = 0, st_cells = 0, st_table = 0, st_tb = 0, st_steps = 0;
    const uint64_t rorg = P.planes_from_off0 ? (P.read_off[0] & ~63ull) : 0;
    const uint64_t forg = P.planes_from_off0 ? (P.ref_off[0] & ~63ull) : 0;
    SeqCursor rc, fc;
    seq_open(rc, P.read_lo, P.read_hi, pc.rb - rorg);
    seq_open(fc, P.ref_lo, P.ref_hi, pc.fb - forg + ti);
    const uint32_t max_windows = (uint32_t)pc.m + (uint32_t)pc.n + 1u;
    const int K = P.K;  // rows 0..K, K <= 64
    const int d = lane;
    while (pj < pc.m) {
        if (nwin >= max_windows) { failed = internal = true; break; }
        const int mw = min(P.W, pc.m - pj);
        const int nw = min(P.W, pc.n - ti);
        ++nwin;
        u64 pl, ph, tl, th;
        seq_window(rc, P.read_lo, P.read_hi, pc.rb - rorg + pj, pl, ph);
        seq_window(fc, P.ref_lo, P.ref_hi, pc.fb - forg + ti, tl, th);
        u64 pm[4];
        pm_from_planes(pl, ph, mw, pm);
        store_pmt<64>(smem, lane, pm, tl, th, nw);
        wave_sync();
        // DC over all rows and columns
        const u64* pmt = smem + OFF_PMT;
        u64 R = init_word(d);
        u64 Dp = d == 0 ? ~0ull : init_word(d - 1);
        u64 R64 = 0ull;  // row 64 (lane 63, K = 64): init word 0
        u64 col0 = R, col0_64 = R64;
        for (int t = 0; t < nw + 63; ++t) {
            const int i = nw - 1 - t + d;
            const u64 pm_t = pmt[clampi(i, 0, nw)];
            const u64 up = LaneShift<64>::up(~0ull, R);
            const u64 m = (R << 1) | pm_t;
            const u64 sw = Dp << 1, iw = up << 1, dw = Dp;
            const u64 Rn = d == 0 ? m : (m & sw & iw & dw);
            const bool live = i >= 0 && i < nw && d <= K;
            if (live) store_edges(tab + ((size_t)d * 64 + i) * 4, m, sw, iw, dw);
            if (d == 63 && K == 64 && i >= 0 && i < nw) {
                // row 64 from row 63: D = R63[i+1] (R), U = R63[i] (Rn)
                const u64 m64 = (R64 << 1) | pm_t;
                const u64 s64 = R << 1, i64 = Rn << 1, d64 = R;
                store_edges(tab + ((size_t)64 * 64 + i) * 4, m64, s64, i64, d64);
                R64 = m64 & s64 & i64 & d64;
                if (i == 0) col0_64 = R64;
            }
            if (i == 0) col0 = Rn;
            Dp = up;
            R = Rn;
        }
        mem_sync();
        st_cells += (u64)mw * nw;
        st_steps += 64ull * (nw + 63);
        int dstar = -1;
        if (nw == 0) {
            // no columns: every row holds its initial word
            col0 = init_word(d);
            col0_64 = 0ull;
        }
        const bool sol = d <= K && !((col0 >> (mw - 1)) & 1ull);
        const u64 bits = __ballot(sol);
        if (bits) dstar = __builtin_ctzll(bits);
        else if (K == 64) {
            const u64 b64 = __ballot(lane == 63 && !((col0_64 >> (mw - 1)) & 1ull));
            if (b64) dstar = 64;
        }
        if (dstar < 0) { failed = true; break; }
        TbOut t;
        run_window_start(runs, rs, writer);
        t = traceback_unimproved(tab, runs, rs, writer, pl, ph, tl, th, mw, nw, dstar, P.L, internal);
        if (internal) { failed = true; break; }
        score += t.edits;
        st_tb += t.reads;
        st_wops += (u64)nw * (2 + 6 * (u64)K);
        st_table += (u64)nw * (4ull * (K + 1) - 3);
        wave_sync();
        const int closed = max(rs.nr, 0);
        overflow |= copy_runs<64>(runs, closed, P.cigar, run_base, run_limit, written, lane);
        written += (uint32_t)closed;
        wave_sync();
        ti += t.i_end;
        pj += t.j_end;
    }
    if (!failed && writer && rs.cur_op >= 0) {
        const uint64_t idx = run_base + written;
        if (idx < run_limit) P.cigar[idx] = (rs.cur_len << 2) | (uint32_t)rs.cur_op;
        else overflow = true;
    }
    const bool ovf = __ballot(overflow) != 0;
    if (lane == 0) {
        genasm_result r;
        if (failed) {
            r.edit_distance = -1;
            r.ref_begin = r.ref_end = 0;
            r.cigar_len = 0;
        } else {
            r.edit_distance = score;
            r.ref_begin = (uint32_t)col;
            r.ref_end = (uint32_t)ti;
            r.cigar_len = ovf ? 0u : written + (rs.cur_op >= 0 ? 1u : 0u);
        }
        r.n_windows = nwin;
        r.cigar_off = run_base;
        r.flags = (ovf && !failed ? GENASM_FLAG_CIGAR_OVERFLOW : 0u) |
                  (internal ? GENASM_FLAG_INTERNAL : 0u);
        P.out[pair] = r;
        if (P.stats) {
            u64* stp = P.stats + pair * kStatCount;
            stp[kStatWindowWordOps] += st_wops;
            stp[kStatWindowCells] += st_cells;
            stp[kStatTableWords] += st_table;
            stp[kStatTbReads] += st_tb;
            stp[kStatWindowLaneSteps] += st_steps;
            stp[kStatWindows] += nwin;
        }
    }
}

// ---------------------------------------------------------------------------
// Batched form: start search with a retry list, then a persistent window kernel
// ---------------------------------------------------------------------------

// Pops one item per group from a device queue; returns the same value in all
// lanes of the group.
// Once the list is drained a plain load of the head says so, and the group
// returns without an atomic: thousands of groups finding an empty list would
// otherwise serialize on the one counter (tens of microseconds per launch).
__device__ __forceinline__ uint32_t group_pop(uint32_t* head, u64* lds, int gl, uint32_t n) {
    if (gl == 0) {
        uint32_t v = __hip_atomic_load(head, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (v < n) v = atomicAdd(head, 1u);
        lds[OFF_BC + 3] = v;
    }
    wave_sync();
    const uint32_t v = (uint32_t)lds[OFF_BC + 3];
    wave_sync();
    return v;
}

// Start search over reference chunks. An item is (pair, chunk): chunk c's
// output columns are [cC, min(n, (c+1)C)) for C = search_chunk (the whole
// reference when 0). R[d][i] depends only on T[i .. i + m1 + d), so the chunk
// scans its output columns plus the next m1 + 64 columns with the text end put
// there, which gives exactly the full-reference values on its output columns.
// Each chunk's least hit row and leftmost hit column go into the pair's key
// (row << 32 | column) by an atomic minimum; the least key over the chunks is
// the full search's answer (least row, then leftmost column).
__device__ __forceinline__ uint32_t search_pairs(const AlignParams& P) {
    return P.list_in ? __hip_atomic_load(P.counters + kCounterPairs, __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT)
                     : (uint32_t)P.n_pairs;
}

__device__ __forceinline__ uint32_t search_chunks(const AlignParams& P, int n) {
    return P.search_chunk ? max(1u, ((uint32_t)n + P.search_chunk - 1) / P.search_chunk) : 1u;
}

// One thread per pair of the list (or of the batch): clears the pair's key and
// appends its chunk items to the stage-0 item list.
__global__ void k_search_items(AlignParams P) {
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t n_items = search_pairs(P);
    if (k >= n_items) return;
    const uint64_t pair = P.list_in ? P.list_in[k] : k;
    P.search_key[pair] = ~0ull;
    const PairCursor pc = pair_cursor(P, pair);
    if (pc.m == 0) return;  // settled by the finalize kernel
    const uint32_t nc = search_chunks(P, pc.n);
    const uint32_t at = atomicAdd(P.counters + kCounterListBase, nc);
    for (uint32_t c = 0; c < nc; ++c) P.items_out[at + c] = (pair << 24) | c;
}

template <int G, int RS>
__global__ __launch_bounds__(64) void k_search(AlignParams P) {
    extern __shared__ u64 smem[];
    const int lane = threadIdx.x & 63;
    const int gl = lane & (G - 1);
    u64* lds = smem + (threadIdx.x / G) * kSearchGroupWords;
    uint32_t* len_in = P.counters + kCounterListBase + 2 * P.list_slot;
    uint32_t* head = len_in + 1;
    uint32_t* len_out = len_in + 2;
    const uint32_t n_items = __hip_atomic_load(len_in, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const int rows_before = P.list_slot == 0 ? 0 : (P.list_slot == 1 ? 16 : 32);
    // A group takes at most n_items items, which bounds the loop.
    for (uint32_t iter = 0; iter <= n_items; ++iter) {
        const uint32_t item = group_pop(head, lds, gl, n_items);
        if (item >= n_items) break;
        const uint64_t it = P.items_in[item];
        const uint64_t pair = it >> 24;
        const uint32_t chunk = (uint32_t)(it & 0xffffffull);
        if (rows_before && (P.search_key[pair] >> 32) < (uint64_t)rows_before)
            continue;  // an earlier stage already found the pair's least row
        const PairCursor pc = pair_cursor(P, pair);
        const int m1 = min(P.W, pc.m);
        const int Kr = min(P.K, m1 - 1);
        const int c0 = P.search_chunk ? (int)(chunk * P.search_chunk) : 0;
        const int c1 = P.search_chunk ? min(pc.n, c0 + (int)P.search_chunk) : pc.n;
        const int e = min(pc.n, c1 + m1 + 64);
        build_pm<G>(lds, gl, P.reads, pc.rb, m1, false);
        int row, col;
        search_rows<G, RS>(lds, gl, lane, P.refs, pc.fb + c0, e - c0, m1, Kr, &row, &col, c1 - c0);
        if (gl == 0) {
            if (P.stats)
                atomicAdd(P.stats + pair * kStatCount + kStatSearchLaneSteps,
                          (u64)G * RS * (u64)(e - c0 + RS * G - 1));
            if (row >= 0) {
                atomicMin(P.search_key + pair, ((u64)(unsigned)row << 32) | (u64)(unsigned)(c0 + col));
            } else if (Kr >= RS * G) {
                const uint32_t pos = atomicAdd(len_out, 1u);
                P.items_out[pos] = it;
            }
        }
    }
}

// The search outcome of one pair from its key: ends the pairs that need no
// window (empty read: score 0; no hit within K rows: -1) and returns the start
// row of the others (-1 for the ended ones).
__device__ int search_outcome(const AlignParams& P, uint64_t pair) {
    const PairCursor pc = pair_cursor(P, pair);
    if (pc.m == 0) {
        finish_without_windows(P, pair, 0);
        P.search[pair] = SearchOut{kSearchDone, 0};
        return -1;
    }
    const int m1 = min(P.W, pc.m);
    const u64 key = P.search_key[pair];
    int row, col;
    if (key != ~0ull) {
        row = (int)(key >> 32);
        col = (int)(uint32_t)key;
    } else if (m1 <= P.K) {
        row = m1;  // row m1 hits in every column
        col = 0;
    } else {
        row = -1;
        col = 0;
    }
    if (P.stats) {
        u64* st = P.stats + pair * kStatCount;
        st[kStatSearchWordOps] = (u64)pc.n * (2 + 6 * (u64)(row >= 0 ? row : min(P.K, m1 - 1)));
        st[kStatSearchCells] = (u64)m1 * pc.n;
    }
    if (row < 0) {
        finish_without_windows(P, pair, -1);
        P.search[pair] = SearchOut{kSearchFailed, 0};
        return -1;
    }
    P.search[pair] = SearchOut{row, (uint32_t)col};
    return row;
}

// Appends the calling lanes with `want` set to a device list with one atomic
// per wavefront; returns each such lane's position.
__device__ __forceinline__ uint32_t wave_append(uint32_t* len, bool want) {
    const u64 bits = __ballot(want);
    const int lane = threadIdx.x & 63;
    const int leader = bits ? __builtin_ctzll(bits) : 0;
    uint32_t base = 0;
    if (want && lane == leader) base = atomicAdd(len, (uint32_t)__builtin_popcountll(bits));
    base = __shfl(base, leader);
    return base + (uint32_t)__builtin_popcountll(bits & ((1ull << lane) - 1ull));
}

// One thread per pair of the list (or of the batch): the pair's search outcome,
// then its window queue (one device atomic per wavefront and queue).
__global__ void k_search_finalize(AlignParams P) {
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t n_items = search_pairs(P);
    bool easy = false, hard = false, ended = false;
    uint64_t pair = 0;
    if (k < n_items) {
        pair = P.list_in ? P.list_in[k] : k;
        const int row = search_outcome(P, pair);
        if (row >= 0 && P.route) {
            hard = row >= P.hard_row;
            easy = !hard;
        }
        ended = row < 0;
    }
    if (P.fin_list) {
        // serving: a pair that ends in its search (empty read, no hit) is finished
        const uint32_t pf = wave_append(P.fin_len, ended);
        if (ended) P.fin_list[pf] = (uint32_t)pair;
    }
    if (!P.route) return;
    const uint32_t pe = wave_append(P.counters + kCounterEasyLen, easy);
    const uint32_t ph = wave_append(P.counters + kCounterHardLen, hard);
    if (easy) P.easy_list[pe] = (uint32_t)pair;
    if (hard) P.hard_list[ph] = (uint32_t)pair;
}

// Window kernel of the batched form. Each workgroup is one wavefront. Pairs
// come from two queues filled by the start search: the hard queue (start row
// >= hard_row: decoy-like pairs whose windows need several DC passes) and the
// easy queue. A share of the workers drains the hard queue first, so that the
// costliest pairs start early and the queue tail is made of cheap ones, while
// the rest start on the easy queue: hard pairs spill table rows to device
// memory, and fewer of them at a time keeps that traffic in the caches. With hard_lanes
// 64 a hard pair takes a whole wavefront (all 64 rows in one pass, the full
// table in LDS); with 32, half a wavefront (32 rows per pass, 32 rows in LDS);
// otherwise, and always for the easy queue, every pair runs in a 16-lane group,
// four pairs per wavefront, with `lds_rows` table rows in LDS and the rows
// above spilled to device memory.
//
// HL, the hard queue's group width (16, 32 or 64), is a template argument so
// that each instance holds only the paths its launch runs (the widest path
// sets the register allocation of the whole kernel).
template <int HL>
__global__ __launch_bounds__(64) void k_windows(AlignParams P) {
    extern __shared__ u64 smem[];
    const int lane = threadIdx.x & 63;
    const uint32_t n_hard = __hip_atomic_load(P.counters + kCounterHardLen, __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT);
    const uint32_t n_easy = __hip_atomic_load(P.counters + kCounterEasyLen, __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT);
    // the first hard_share percent of the workgroups (spread over the CUs by the
    // dispatch order) drain the hard queue first, the others the easy queue
    const bool hard_first = (uint64_t)blockIdx.x * 100u < (uint64_t)gridDim.x * (uint32_t)P.hard_share;
    const int gl = lane & 15;
    const int grp = lane >> 4;
    u64* lds = smem + grp * window_group_words(P.lds_rows, P.stride);
    const int spill_rows = 64 - P.lds_rows;
    u64* spill = spill_rows > 0
        ? P.spill + ((uint64_t)blockIdx.x * 4 + grp) * (uint64_t)spill_group_words(spill_rows) : nullptr;
    for (int phase = 0; phase < 2; ++phase) {
        const bool hard = (phase == 0) == hard_first;
        if (HL == 64 && hard) {
            for (uint32_t iter = 0; iter <= n_hard; ++iter) {
                const uint32_t item = group_pop(P.counters + kCounterHardHead, smem, lane, n_hard);
                if (item >= n_hard) break;
                const uint64_t pair = P.hard_list[item];
                const SearchOut so = P.search[pair];
                if (so.row < 0) continue;  // ended in the search (result already written)
                run_pair<64>(P, smem, nullptr, 64, lane, lane, pair, (int)so.col);
            }
            continue;
        }
        if (HL == 32 && hard) {
            // two 32-lane groups, each with 32 table rows in LDS (the space of two
            // 16-lane groups) and rows 32..63 (one spilled pass) in the spill
            // areas of those two groups (each at least half a 32-lane block; a
            // 16-lane group spills when lds_rows <= 48, the limit for this form)
            const int gl32 = lane & 31;
            const int h = lane >> 5;
            u64* lds32 = smem + h * window_group_words32(32, P.stride);
            u64* spill32 = P.spill + ((uint64_t)blockIdx.x * 4 + 2 * h) *
                                         (uint64_t)spill_group_words(64 - P.lds_rows);
            for (uint32_t iter = 0; iter <= n_hard; ++iter) {
                const uint32_t item = group_pop(P.counters + kCounterHardHead, lds32, gl32, n_hard);
                if (item >= n_hard) break;
                const uint64_t pair = P.hard_list[item];
                const SearchOut so = P.search[pair];
                if (so.row < 0) continue;  // ended in the search (result already written)
                run_pair<32>(P, lds32, spill32, 32, gl32, lane, pair, (int)so.col);
            }
            continue;
        }
        const uint32_t* list = hard ? P.hard_list : P.easy_list;
        const uint32_t n = hard ? n_hard : n_easy;
        uint32_t* head = P.counters + (hard ? kCounterHardHead : kCounterEasyHead);
        for (uint32_t iter = 0; iter <= n; ++iter) {
            const uint32_t item = group_pop(head, lds, gl, n);
            if (item >= n) break;
            const uint64_t pair = list[item];
            const SearchOut so = P.search[pair];
            if (so.row < 0) continue;  // ended in the search (result already written)
            run_pair<16>(P, lds, spill, P.lds_rows, gl, lane, pair, (int)so.col);
        }
    }
}

// ---------------------------------------------------------------------------
// Compact window groups: 16 lanes, the table in LDS as 32-bit slices
// ---------------------------------------------------------------------------
//
// The traceback of a window reads, at an edit from state (i, j, d), bits p-1
// and p of R[d-1][i+1] and bit p-1 of R[d-1][i], with p = mw-1-j. Every edit
// moves the diagonal i - j by at most one, so after d*-d edits |i - j| <=
// d*-d: the bits the traceback can ever read from entry (r, c) lie within
// d*-r positions of bit mw-1-c. When d* <= 15 that is a 32-bit window, and
// the table can keep 32 bits per entry instead of 64.
//
// The pass runs in aligned form: every word shifted left by a = 64 - mw, so
// that the first pattern base is bit 63 whatever mw is (the recurrence is
// unchanged under the shift: the row above row 0 is all ones, the bit that
// row 0 adds is 1 << a, the initial column is (~0 << d) << a, and PM is
// shifted likewise; bits below a stay zero). Entry (r, c) keeps the 32 bits
// of the aligned word from bit o(c) = max(0, 47-c) on: the traceback's bits
// 62-j (and 63-j) then sit at 62-j-o(c) (63-j-o(c)), which with |i - j| <= 14
// is in 0..31 (15+e at column i and 16+e, 17+e at column i+1 for columns up
// to 47, e = i - j). Columns past 47 occur only when W-O > 47.
//
// Layout of a compact group (64-bit words): the step-ordered PM[T] array at
// words 0..78 (kCompactPmt + x for x in -15..63; the traceback's run records
// reuse it), then 16 table rows of `stride` 32-bit slots from word
// kCompactTab (slot 0 and slot W-O+2 of a row are dummies, as in the 64-bit
// table). A window that needs more than 16 rows (a deep window) is computed
// again with 64-bit rows, all of them in the group's spill area in device
// memory, using the 16-lane code of the 64-bit layout: its boundary row and
// run records then sit in the table area, at the same offsets as there.
constexpr int kCompactPmt = 15;
constexpr int kCompactTab = 79;
constexpr int kCompactRows = 16;
constexpr int kCompactU = 4;  // DC steps per unrolled chunk (compact and deep passes)
static_assert(kCompactSpillRows == 64, "a deep window may need every row");
static_assert(kCompactTab == kCompactPmt + 64, "layout");
// Words the deep (64-bit, spilled) passes use past the PM[T] array: the
// boundary row at SoLayout<16>::brow = 94 with reads up to word 94 + nw + 13
// + 2U, and the run records at 94..157.
constexpr int kCompactDeepWords = OFF_BROW16 + 64 + 13 + 2 * kCompactU + 1;

__host__ __device__ inline int compact_group_words(int stride) {
    const int tab = kCompactTab + (kCompactRows * stride + 1 + 1) / 2;
    return tab > kCompactDeepWords ? tab : kCompactDeepWords;
}

// Aligned initial word of row d: (~0 << d) << a.
__device__ __forceinline__ u64 init_word_a(int d, int a) { return d + a >= 64 ? 0ull : (~0ull << (d + a)); }

// Slice offset o(c) of the compact table (see above).
__device__ __forceinline__ int slice_off(int c) { return max(0, 47 - c); }

// Pass 0 of a window in aligned form (this lane: row gl), storing each
// entry's 32-bit slice (slot 1 + c of row gl; steps outside columns 0..Lc
// store into the dummies, and the leading steps whose columns all lie past
// Lc store nothing). WIDE: stored columns may pass 47 (W-O > 47), so the
// slice offset needs its clamp at zero.
template <bool WIDE>
__device__ __forceinline__ void dc_pass_c(u64* lds, int gl, int nw, int Lc, int stride, int a) {
    uint32_t* trow = reinterpret_cast<uint32_t*>(lds + kCompactTab) + gl * stride;
    const u64* pp = lds + kCompactPmt - gl;  // + t: PMT[t - gl]
    u64 R = init_word_a(gl, a);
    u64 Dp = gl == 0 ? ~0ull : init_word_a(gl - 1, a);
    const u64 lowin = gl == 0 ? (1ull << a) : 0ull;
    if (Lc == nw) trow[1 + nw] = (uint32_t)(R >> slice_off(nw));  // column nw: the initial word
    const int slot0 = nw + gl;      // slot 1 + i at t = 0 (column i = nw - 1 - t + gl)
    const int sh0 = 48 - nw - gl;   // 47 - i at t = 0
    const int hi_slot = Lc + 2;
    const int steps = nw + 15;
    constexpr int U = kCompactU;
    u64 qpm[U];
#pragma unroll
    for (int u = 0; u < U; ++u) qpm[u] = pp[u];
    auto chunk = [&](int t0, auto store) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int t = t0 + u;
            const u64 pm_t = qpm[u];
            const u64 up = shift_up<16>(~0ull, R, gl);
            R = dc_step(R, Dp, up, pm_t, lowin);
            Dp = up;
            if constexpr (decltype(store)::value) {
                // live stores have 47 - i <= 47; the dummies store garbage
                const int sh = WIDE ? max(0, sh0 + t) : sh0 + t;
                trow[med3i(slot0 - t, 0, hi_slot)] = (uint32_t)(R >> (sh & 63));
            }
            if (u & 1) {
                qpm[u - 1] = pp[t - 1 + U];
                qpm[u] = pp[t + U];
            }
        }
    };
    using yes = std::integral_constant<bool, true>;
    using no = std::integral_constant<bool, false>;
    const int t_free = nw - Lc - 1;
    int t0 = 0;
    for (; t0 + U <= t_free; t0 += U) chunk(t0, no{});
    for (; t0 < steps; t0 += U) chunk(t0, yes{});
}

// Traceback of a compact window (d* <= 15): traceback_planes with the edge
// bits taken from the 32-bit slices.
__device__ __forceinline__ TbOut traceback_c(const u64* lds, uint32_t* runs, RunState& rs, u64 pl,
                                             u64 ph, u64 tl, u64 th, int mw, int nw, int dstar, int L,
                                             int stride) {
    const uint32_t* tab = reinterpret_cast<const uint32_t*>(lds + kCompactTab) + 1;
    const int jmax = min(mw, L);
    int i = 0, j = 0, d = dstar;
    TbOut o{0, 0, 0, 0u, false};
    for (int it = 0; it <= 2 * L; ++it) {
        if (j >= jmax || i >= L) break;
        const u64 mis = ((pl >> j) ^ (tl >> i)) | ((ph >> j) ^ (th >> i));
        const int k = min(ctz64(mis), min(jmax - j, min(L - i, nw - i)));
        {
            const bool push = k > 0;
            const bool changed = push && rs.cur_op != (int)GENASM_OP_MATCH;
            rs.nr += changed ? 1 : 0;
            rs.cur_len = changed ? (uint32_t)k : rs.cur_len + (uint32_t)k;
            rs.cur_op = push ? (int)GENASM_OP_MATCH : rs.cur_op;
            runs[max(rs.nr, 0)] = (rs.cur_len << 2) | (uint32_t)rs.cur_op;
            i += k;
            j += k;
            if (j >= jmax || i >= L) break;
        }
        if (d < 1) { o.internal = true; break; }
        const uint32_t* row = tab + (d - 1) * stride;
        const uint32_t C = row[i];
        const uint32_t B = row[i + 1];
        const int kc = 62 - j - slice_off(i);      // bit p-1 of R[d-1][i]
        const int kb = 62 - j - slice_off(i + 1);  // bit p-1 of R[d-1][i+1]; bit p is kb + 1
        const bool intext = i < nw;
        const bool s_ok = intext && !((B >> kb) & 1u);
        const bool i_ok = !((C >> kc) & 1u);
        const bool d_ok = intext && !((B >> (kb + 1)) & 1u);
        if (!(s_ok || i_ok || d_ok)) { o.internal = true; break; }
        const int op = s_ok ? GENASM_OP_MISMATCH : i_ok ? GENASM_OP_INS : GENASM_OP_DEL;
        run_push(runs, rs, op, 1u, true);
        o.reads += 2u;
        i += op != GENASM_OP_INS;
        j += op != GENASM_OP_DEL;
        d -= 1;
    }
    o.i_end = i;
    o.j_end = j;
    o.edits = dstar - d;
    return o;
}

// advance_pair for compact groups. A window first runs the compact pass
// (unless the pair's previous window was deep); when no row below 16 solves,
// it is computed again with 64-bit rows in the spill area (every row, in
// passes of 16) and traced back from there. STATS: profiling counters.
template <bool STATS>
__device__ __forceinline__ uint32_t advance_pair_c(const AlignParams& P, u64* lds, u64* spill, int gl,
                                                   int lane, uint64_t pair, const PairCursor& pc,
                                                   int s, PairState& st, uint32_t budget,
                                                   TurnClock& turn) {
    constexpr int G = 16;
    const uint64_t run_base = pair_run_base(P, pair);
    const uint64_t run_limit = min(P.cigar_cap, run_base + (uint64_t)pc.m + (uint64_t)pc.n);
    uint32_t* runs_c = reinterpret_cast<uint32_t*>(lds);               // PM[T] area, free after the pass
    uint32_t* runs_d = reinterpret_cast<uint32_t*>(lds + OFF_RUNS16);  // deep windows
    RunState rs{st.cur_op, st.cur_len, st.cur_op >= 0 ? 0 : -1};
    bool overflow = (st.flags & kStateOverflow) != 0;
    bool deep = (st.flags & kStateDeep) != 0;
    bool failed = false, internal = false;
    u64 st_wops = 0, st_cells = 0, st_table = 0, st_tb = 0, st_steps = 0;
    u64 cyc_dc = 0, cyc_tb = 0, cyc_start = 0, wall_start = 0;
    if constexpr (STATS) {
        cyc_start = clock64();
        wall_start = wall_clock64();
    }
    const uint32_t max_windows = (uint32_t)pc.m + (uint32_t)pc.n + 1u;
    uint32_t done_here = 0;
    const uint64_t rorg = P.planes_from_off0 ? (P.read_off[0] & ~63ull) : 0;
    const uint64_t forg = P.planes_from_off0 ? (P.ref_off[0] & ~63ull) : 0;
    SeqCursor rc, fc;
    if (st.pj < pc.m) {
        seq_open(rc, P.read_lo, P.read_hi, pc.rb - rorg + st.pj);
        seq_open(fc, P.ref_lo, P.ref_hi, pc.fb - forg + st.ti);
    }
    while (st.pj < pc.m && (budget == 0 || done_here < budget)) {
        // see advance_pair: at least one window per launch, none once the turn has ended
        if (turn.active && done_here > 0 && turn.over()) break;
        if (st.nwin >= max_windows) { failed = true; internal = true; break; }
        const int mw = min(P.W, pc.m - st.pj);
        const int nw = min(P.W, pc.n - st.ti);
        const int Lc = min(nw, P.L);
        ++st.nwin;
        ++done_here;
        u64 cyc0 = 0;
        if constexpr (STATS) cyc0 = clock64();
        u64 pl, ph, tl, th;
        seq_window(rc, P.read_lo, P.read_hi, pc.rb - rorg + st.pj, pl, ph);
        seq_window(fc, P.ref_lo, P.ref_hi, pc.fb - forg + st.ti, tl, th);
        const int Kr = nw > 0 ? min(P.K, mw - 1) : -1;
        int dstar = -1;
        bool compact = false;
        if constexpr (STATS) st_cells += (u64)mw * nw;
        if (Kr >= 0) {
            u64 pm[4];
            pm_from_planes(pl, ph, mw, pm);
            if (!deep) {
                const int a = 64 - mw;
                const u64 pma[4] = {pm[0] << a, pm[1] << a, pm[2] << a, pm[3] << a};
                store_pmt_so<G>(lds, gl, pma, tl, th, nw);
                wave_sync();
                if constexpr (STATS) st_steps += (u64)G * (nw + G - 1);
                if (P.L > 47) dc_pass_c<true>(lds, gl, nw, Lc, P.stride, a);
                else dc_pass_c<false>(lds, gl, nw, Lc, P.stride, a);
                wave_sync();
                const uint32_t s0 = reinterpret_cast<const uint32_t*>(lds + kCompactTab)[gl * P.stride + 1];
                const bool sol = gl <= Kr && !((s0 >> 16) & 1u);  // bit 63 of the aligned word
                const u64 bits = group_ballot(sol, G, lane);
                if (bits) {
                    dstar = __builtin_ctzll(bits);
                } else if (Kr < G) {
                    // every row that needs computing was computed: row mw solves
                    if (mw <= P.K) dstar = mw;
                    else { failed = true; break; }
                }
                compact = dstar >= 0 && dstar < G;
            }
            if (!compact) {
                // deep window: every row again, 64-bit, in the spill area
                store_pmt_so<G>(lds, gl, pm, tl, th, nw);
                wave_sync();
                dstar = -1;
                for (int c = 0; c * G <= Kr; ++c) {
                    if constexpr (STATS) st_steps += (u64)G * (nw + G - 1);
                    if (c == 0) {
                        dc_pass_so<G, true, true, kCompactU>(lds, spill, gl, c, nw, Lc, P.stride, 0);
                    } else {
                        fill_brow<G>(lds, spill, gl, c, nw, Lc, P.stride, 0);
                        wave_sync();
                        dc_pass_so<G, true, false, kCompactU>(lds, spill, gl, c, nw, Lc, P.stride, 0);
                    }
                    mem_sync();
                    const int d = c * G + gl;
                    const u64 r0 = load_spill(spill_entry<G>(spill, d, 0, nw, 0));
                    const bool sol = d <= Kr && !((r0 >> (mw - 1)) & 1ull);
                    const u64 bits = group_ballot(sol, G, lane);
                    if (bits) { dstar = c * G + __builtin_ctzll(bits); break; }
                }
                if (dstar < 0) {
                    if (mw <= P.K) dstar = mw;
                    else { failed = true; break; }
                }
            }
        }
        u64 cyc1 = 0;
        if constexpr (STATS) cyc1 = clock64();
        TbOut t;
        uint32_t* runs = compact || nw == 0 ? runs_c : runs_d;
        run_window_start(runs, rs, true);
        if (nw == 0) {
            const int k = min(mw, P.L);
            run_push(runs, rs, GENASM_OP_INS, (uint32_t)k, true);
            t = TbOut{0, k, k, 0u, false};
        } else if (compact) {
            t = traceback_c(lds, runs, rs, pl, ph, tl, th, mw, nw, dstar, P.L, P.stride);
        } else {
            t = traceback_planes<G>(lds, spill, runs, rs, true, pl, ph, tl, th, mw, nw, dstar, P.L,
                                    P.stride, 0, gl, lane, P.tb_prefetch != 0);
        }
        // the next window starts deep when this one needed more than 16 rows
        if (nw > 0) deep = dstar >= G;
        st.score += t.edits;
        if constexpr (STATS) {
            st_tb += t.reads;
            st_wops += (u64)nw * (2 + 6 * dstar);
            st_table += (u64)(dstar + 1) * (Lc + 1);
        }
        if (t.internal) { failed = true; internal = true; break; }
        wave_sync();
        const int closed = max(rs.nr, 0);
        overflow |= copy_runs<G>(runs, closed, P.cigar, run_base, run_limit, st.written, gl);
        st.written += (uint32_t)closed;
        wave_sync();
        st.ti += t.i_end;
        st.pj += t.j_end;
        if constexpr (STATS) {
            const u64 cyc2 = clock64();
            cyc_dc += cyc1 - cyc0;
            cyc_tb += cyc2 - cyc1;
        }
    }
    st.cur_op = rs.cur_op;
    st.cur_len = rs.cur_len;
    st.flags = deep ? (st.flags | kStateDeep) : (st.flags & ~kStateDeep);
    const bool finished = failed || st.pj >= pc.m;
    if (finished && !failed && gl == 0 && rs.cur_op >= 0) {
        const uint64_t idx = run_base + st.written;
        if (idx < run_limit) P.cigar[idx] = (rs.cur_len << 2) | (uint32_t)rs.cur_op;
        else overflow = true;
    }
    if (group_ballot(overflow, G, lane) != 0) st.flags |= kStateOverflow;
    if (failed) st.flags |= kStateFailed;
    if (internal) st.flags |= kStateInternal;
    if (finished) st.flags |= kStateDone;
    if (gl == 0 && finished) {
        const bool ovf = (st.flags & kStateOverflow) != 0;
        genasm_result r;
        if (failed) {
            r.edit_distance = -1;
            r.ref_begin = r.ref_end = 0;
            r.cigar_len = 0;
        } else {
            r.edit_distance = st.score;
            r.ref_begin = (uint32_t)s;
            r.ref_end = (uint32_t)st.ti;
            r.cigar_len = ovf ? 0u : st.written + (rs.cur_op >= 0 ? 1u : 0u);
        }
        r.n_windows = st.nwin;
        r.cigar_off = run_base;
        r.flags = (ovf && !failed ? GENASM_FLAG_CIGAR_OVERFLOW : 0u) |
                  (internal ? GENASM_FLAG_INTERNAL : 0u);
        P.out[pair] = r;
    }
    if constexpr (STATS) {
        if (gl == 0) {
            u64* stp = P.stats + pair * kStatCount;
            stp[kStatWindowWordOps] += st_wops;
            stp[kStatWindowCells] += st_cells;
            stp[kStatTableWords] += st_table;
            stp[kStatTbReads] += st_tb;
            stp[kStatWindowLaneSteps] += st_steps;
            stp[kStatWindows] += done_here;
            stp[kStatDcCycles] += cyc_dc;
            stp[kStatTbCycles] += cyc_tb;
            stp[kStatPairCycles] += clock64() - cyc_start;
            if (!stp[kStatPairStart]) stp[kStatPairStart] = wall_start;
            stp[kStatPairEnd] = wall_clock64();
        }
    }
    return done_here;
}

// run_pair for compact groups; `deep_start`: the pair came from the hard
// queue, so its first window starts deep.
template <bool STATS>
__device__ __forceinline__ void run_pair_c(const AlignParams& P, u64* lds, u64* spill, int gl, int lane,
                                           uint64_t pair, int s, bool deep_start) {
#if defined(GENASM_DEBUG)
    if (P.audit && gl == 0) atomicAdd(P.audit + pair, kAuditTake);  // queue audit
#endif
    const PairCursor pc = pair_cursor(P, pair);
    if (!P.state) {
        PairState st = fresh_state(s);
        if (deep_start) st.flags |= kStateDeep;
        TurnClock none;
        advance_pair_c<STATS>(P, lds, spill, gl, lane, pair, pc, s, st, 0u, none);
        return;
    }
    PairState st = P.state[pair];
    if (st.flags & kStateDone) return;
    if (!(st.flags & kStateStarted)) st = fresh_state(s);
    TurnClock turn;
    turn.open(P);
    const uint32_t advanced =
        advance_pair_c<STATS>(P, lds, spill, gl, lane, pair, pc, s, st, P.window_budget, turn);
    if (gl == 0) {
        P.state[pair] = st;
        if (P.fin_list) {
            if (st.flags & kStateDone)
                P.fin_list[atomicAdd(P.fin_len, 1u)] = (uint32_t)pair;
            else if (advanced <= 1)
                P.next_hot[atomicAdd(P.next_len + kCounterEasyLen, 1u)] = (uint32_t)pair;
            else
                P.next_cold[atomicAdd(P.next_len + kCounterHardLen, 1u)] = (uint32_t)pair;
        }
    }
}

// Window kernel with compact groups (four 16-lane groups per wavefront, both
// queues; see k_windows for the queues and the hard share). Each group's
// spill area holds the four step-ordered blocks of a deep window's 64 rows.
template <bool STATS>
__global__ __launch_bounds__(64) void k_windows_c(AlignParams P) {
    extern __shared__ u64 smem[];
    const int lane = threadIdx.x & 63;
    const uint32_t n_hard = __hip_atomic_load(P.counters + kCounterHardLen, __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT);
    const uint32_t n_easy = __hip_atomic_load(P.counters + kCounterEasyLen, __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT);
    const bool hard_first = (uint64_t)blockIdx.x * 100u < (uint64_t)gridDim.x * (uint32_t)P.hard_share;
    const int gl = lane & 15;
    const int grp = lane >> 4;
    u64* lds = smem + grp * compact_group_words(P.stride);
    u64* spill = P.spill + ((uint64_t)blockIdx.x * 4 + grp) * (uint64_t)spill_group_words(kCompactSpillRows);
    for (int phase = 0; phase < 2; ++phase) {
        const bool hard = (phase == 0) == hard_first;
        const uint32_t* list = hard ? P.hard_list : P.easy_list;
        const uint32_t n = hard ? n_hard : n_easy;
        uint32_t* head = P.counters + (hard ? kCounterHardHead : kCounterEasyHead);
        for (uint32_t iter = 0; iter <= n; ++iter) {
            const uint32_t item = group_pop(head, lds, gl, n);
            if (item >= n) break;
            const uint64_t pair = list[item];
            const SearchOut so = P.search[pair];
            if (so.row < 0) continue;  // ended in the search (result already written)
            // serving routes every pair to the easy list; there the hard list
            // holds pairs that already advanced, whose state carries their mode
            run_pair_c<STATS>(P, lds, spill, gl, lane, pair, (int)so.col, hard && !P.state);
        }
    }
}

// ---------------------------------------------------------------------------
// Packing, ordering, compaction
// ---------------------------------------------------------------------------

// 2-bit code of one ASCII base (case folded): A 0, C 1, G 2, T 3, from bits 1
// and 2 of the byte; *ok is false for any other byte (coded 0).
__device__ __forceinline__ unsigned base_code(unsigned ch, bool* ok) {
    ch &= ~0x20u;
    *ok = ch == 'A' || ch == 'C' || ch == 'G' || ch == 'T';
    return *ok ? ((ch >> 1) ^ (ch >> 2)) & 3u : 0u;
}

// Sixteen bases per thread: one 16-byte load, one 4-byte store. Needs `ascii`
// 16-byte aligned and `packed` 4-byte aligned; the last partial chunk takes
// the byte path.
__global__ void k_pack16(const char* ascii, uint64_t n, uint8_t* packed, uint32_t* bad) {
    const uint64_t chunk = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t b0 = chunk * 16;
    if (b0 >= n) return;
    unsigned nbad = 0;
    if (b0 + 16 <= n) {
        const uint4 w = *reinterpret_cast<const uint4*>(ascii + b0);
        const unsigned words[4] = {w.x, w.y, w.z, w.w};
        unsigned out = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                bool ok;
                out |= base_code((words[q] >> (8 * u)) & 0xFFu, &ok) << (8 * q + 2 * u);
                nbad += ok ? 0u : 1u;
            }
        }
        *reinterpret_cast<uint32_t*>(packed + chunk * 4) = out;
    } else {
        for (uint64_t byte = chunk * 4; byte * 4 < n; ++byte) {
            unsigned v = 0;
            for (int u = 0; u < 4; ++u) {
                const uint64_t b = byte * 4 + u;
                if (b < n) {
                    bool ok;
                    v |= base_code((unsigned char)ascii[b], &ok) << (2 * u);
                    nbad += ok ? 0u : 1u;
                }
            }
            packed[byte] = (uint8_t)v;
        }
    }
    if (nbad) atomicAdd(bad, nbad);
}

__global__ void k_pack(const char* ascii, uint64_t n, uint8_t* packed, uint32_t* bad) {
    const uint64_t byte = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (byte * 4 >= n) return;
    unsigned v = 0, nbad = 0;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const uint64_t b = byte * 4 + u;
        if (b < n) {
            const unsigned ch = (unsigned char)ascii[b] & ~0x20u;  // fold case
            unsigned code;
            switch (ch) {
                case 'A': code = 0; break;
                case 'C': code = 1; break;
                case 'G': code = 2; break;
                case 'T': code = 3; break;
                default: code = 0; ++nbad;
            }
            v |= code << (2 * u);
        }
    }
    packed[byte] = (uint8_t)v;
    if (nbad) atomicAdd(bad, nbad);
}

// Resets the queue heads and list lengths; stage 0's list length is set when
// stage 0 walks an explicit list. A kernel rather than a memset so that the
// whole pipeline can be captured in a graph.
__global__ void k_init_counters(uint32_t* counters, uint32_t n_pairs) {
    const int i = threadIdx.x;
    if (i < kCounterCount) counters[i] = i == kCounterPairs ? n_pairs : 0u;
}

__global__ void k_fill_u64(unsigned long long* p, uint64_t n, unsigned long long v) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// Bits 0, 2, 4, ... of x, packed into bits 0..15.
__device__ __forceinline__ uint32_t even_bits(uint32_t x) {
    x &= 0x55555555u;
    x = (x | (x >> 1)) & 0x33333333u;
    x = (x | (x >> 2)) & 0x0F0F0F0Fu;
    x = (x | (x >> 4)) & 0x00FF00FFu;
    x = (x | (x >> 8)) & 0x0000FFFFu;
    return x;
}

// Bases [64w, 64w+64) of a packed stream whose bytes below nbytes may be
// read: four 16-base chunks, bytes at or past nbytes read as 0.
__device__ __forceinline__ void plane_word(const uint8_t* packed, uint64_t nbytes, uint64_t w,
                                           u64& lo, u64& hi) {
    lo = 0;
    hi = 0;
    const uint64_t b0 = w * 16;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        uint32_t x = 0;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const uint64_t b = b0 + 4 * k + u;
            if (b < nbytes) x |= (uint32_t)packed[b] << (8 * u);
        }
        lo |= (u64)even_bits(x) << (16 * k);
        hi |= (u64)even_bits(x >> 1) << (16 * k);
    }
}

// One thread per plane word; see launch_planes.
__global__ void k_planes(const uint8_t* packed, const uint64_t* d_first, uint64_t n_bases, u64* lo,
                         u64* hi, uint64_t nwords) {
    const uint64_t w = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= nwords) return;
    const uint64_t b0 = d_first ? d_first[0] : 0;
    const uint64_t w0 = b0 >> 6;
    u64 a, b;
    plane_word(packed, (b0 + n_bases + 3) / 4, w0 + w, a, b);
    lo[w] = a;
    hi[w] = b;
}

// One block per uploaded range; see launch_scatter_planes.
__global__ void k_scatter_planes(const uint8_t* src, const uint64_t* src_off, const uint32_t* len,
                                 u64* lo, u64* hi, const uint64_t* dst_word, uint32_t n) {
    const uint32_t k = blockIdx.x;
    if (k >= n) return;
    const uint64_t nbytes = ((uint64_t)len[k] + 3) / 4;
    const uint64_t nw = ((uint64_t)len[k] + 63) / 64;
    for (uint64_t w = threadIdx.x; w < nw; w += blockDim.x) {
        u64 a, b;
        plane_word(src + src_off[k], nbytes, w, a, b);
        lo[dst_word[k] + w] = a;
        hi[dst_word[k] + w] = b;
    }
}

// One block per range; see launch_scatter_bytes.
__global__ void k_scatter_bytes(const uint8_t* src, const uint64_t* src_off, uint8_t* dst,
                                const uint64_t* dst_off, const uint32_t* len, uint32_t n) {
    const uint32_t k = blockIdx.x;
    if (k >= n) return;
    const uint8_t* a = src + src_off[k];
    uint8_t* b = dst + dst_off[k];
    for (uint32_t e = threadIdx.x; e < len[k]; e += blockDim.x) b[e] = a[e];
}

// Serving iteration start (one block of 256 threads): counters of this
// iteration and the next, then the admitted requests' slot tables and state.
__global__ void k_serve_begin(uint32_t* cur, uint32_t* next, uint32_t* fin_len,
                              const uint32_t* params, const ServeAdmit* admit, ServeSlots slots,
                              uint32_t* new_list) {
    const uint32_t n_new = params[kServeParamNew];
    const int t = threadIdx.x;
    if (t < kCounterCount) {
        // this iteration's window lists (easy = advanced no window last time,
        // hard = advanced) were filled by the previous iteration: their
        // lengths stay; everything else starts at zero
        if (t != kCounterEasyLen && t != kCounterHardLen) cur[t] = t == kCounterPairs ? n_new : 0u;
        next[t] = 0u;
    }
    if (t == 0) *fin_len = 0u;
    for (uint32_t i = t; i < n_new; i += blockDim.x) {
        const ServeAdmit a = admit[i];
        slots.read_off[a.slot] = a.read_off;
        slots.ref_off[a.slot] = a.ref_off;
        slots.run_base[a.slot] = a.run_base;
        slots.read_len[a.slot] = a.m;
        slots.ref_len[a.slot] = a.n;
        slots.state[a.slot] = PairState{0, 0, 0, 0u, 0u, -1, 0u, 0u};
        new_list[i] = a.slot;
    }
}

__global__ void k_serve_stamp(const uint32_t* params, TurnLimits* turn) {
    const u64 now = wall_clock64();
    const uint32_t ticks = params[kServeParamTicks], soon = params[kServeParamSoonTicks];
    TurnLimits t;
    t.end = ticks ? now + ticks : ~0ull;
    t.soon = soon && (!ticks || soon < ticks) ? now + soon : t.end;
    t.admitted = (u64)params[kServeParamAdmitted] | ((u64)params[kServeParamAdmitted + 1] << 32);
    *turn = t;
}

// Serving iteration end, part 1 (one block of 1024 threads): prefix sum of the
// finished pairs' CIGAR element counts, and the summary the host reads (slot,
// result with cigar_off = the pair's offset in the gathered elements).
__global__ __launch_bounds__(1024) void k_serve_scan(const uint32_t* fin_list, const uint32_t* fin_len,
                                                     const genasm_result* out, uint64_t* fin_off,
                                                     u64* hdr, uint32_t* sum_slot,
                                                     genasm_result* sum_res, uint32_t max_fin) {
    __shared__ u64 part[1024];
    const uint32_t n = min(*fin_len, max_fin);
    const int t = threadIdx.x;
    const uint32_t per = (n + 1023) / 1024;
    const uint32_t lo = min(n, (uint32_t)t * per), hi = min(n, lo + per);
    u64 sum = 0;
    for (uint32_t k = lo; k < hi; ++k) sum += out[fin_list[k]].cigar_len;
    part[t] = sum;
    __syncthreads();
    // inclusive scan of the 1024 partial sums
    for (int d = 1; d < 1024; d <<= 1) {
        const u64 v = t >= d ? part[t - d] : 0ull;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    u64 off = part[t] - sum;
    for (uint32_t k = lo; k < hi; ++k) {
        const uint32_t slot = fin_list[k];
        genasm_result r = out[slot];
        fin_off[k] = off;
        sum_slot[k] = slot;
        r.cigar_off = off;
        sum_res[k] = r;
        off += r.cigar_len;
    }
    if (t == 1023) {
        hdr[0] = n;
        hdr[1] = part[1023];
    }
    __threadfence_system();
}

// Serving iteration end, part 2: the finished pairs' CIGAR elements, pair k at
// dst[fin_off[k]..], for the pairs that fit dst_cap.
__global__ void k_serve_gather(const uint32_t* fin_list, const uint32_t* fin_len,
                               const genasm_result* out, const uint64_t* fin_off,
                               const uint32_t* cigar, uint32_t* dst, uint64_t dst_cap,
                               uint32_t max_fin) {
    const uint32_t n = min(*fin_len, max_fin);
    for (uint32_t k = blockIdx.x; k < n; k += gridDim.x) {
        const genasm_result r = out[fin_list[k]];
        const uint64_t o = fin_off[k];
        if (o + r.cigar_len > dst_cap) continue;
        for (uint32_t e = threadIdx.x; e < r.cigar_len; e += blockDim.x)
            dst[o + e] = cigar[r.cigar_off + e];
    }
}

// Longest-first order by a counting sort over length buckets: bucket 0 holds
// the longest reads. A bucket is the read length's binary exponent and its
// next three bits, so reads within about 12% of each other share a bucket
// (their order inside it is arbitrary; the order only steers scheduling).
__device__ __forceinline__ uint32_t lpt_bucket(uint64_t len) {
    if (len == 0) return kLptBuckets - 1;
    const int e = 63 - __builtin_clzll(len);
    const uint32_t frac = e >= 3 ? (uint32_t)(len >> (e - 3)) & 7u : (uint32_t)(len << (3 - e)) & 7u;
    const uint32_t key = (uint32_t)min(e, 40) * 8u + frac;  // grows with len, < 41 * 8
    return kLptBuckets - 2 - key;
}

// Per-block bucket counts in LDS, then one device atomic per (block, bucket):
// most pairs of a batch share a few buckets, so per-pair device atomics would
// serialize on them.
__global__ void k_lpt_count(const uint64_t* read_off, uint64_t n_pairs, uint32_t* hist) {
    extern __shared__ u64 smem[];
    uint32_t* lh = reinterpret_cast<uint32_t*>(smem);
    for (int t = threadIdx.x; t < kLptBuckets; t += blockDim.x) lh[t] = 0u;
    __syncthreads();
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n_pairs) atomicAdd(&lh[lpt_bucket(read_off[i + 1] - read_off[i])], 1u);
    __syncthreads();
    for (int t = threadIdx.x; t < kLptBuckets; t += blockDim.x)
        if (lh[t]) atomicAdd(&hist[t], lh[t]);
}

// Exclusive prefix sum of the bucket counts, in place (one block of kLptBuckets threads).
__global__ void k_lpt_scan(uint32_t* hist) {
    __shared__ uint32_t v[kLptBuckets];
    const int t = threadIdx.x;
    v[t] = hist[t];
    __syncthreads();
    for (int off = 1; off < kLptBuckets; off <<= 1) {
        const uint32_t x = t >= off ? v[t - off] : 0u;
        __syncthreads();
        v[t] += x;
        __syncthreads();
    }
    hist[t] = t == 0 ? 0u : v[t - 1];
}

// Places pairs at their bucket positions: each block reserves one range per
// bucket it holds (one device atomic per bucket), then numbers its pairs
// inside the ranges with LDS atomics.
__global__ void k_lpt_place(const uint64_t* read_off, uint64_t n_pairs, uint32_t* pos,
                            uint32_t* order) {
    extern __shared__ u64 smem[];
    uint32_t* lh = reinterpret_cast<uint32_t*>(smem);  // counts, then base positions
    uint32_t* lpos = lh + kLptBuckets;
    for (int t = threadIdx.x; t < kLptBuckets; t += blockDim.x) lh[t] = 0u;
    __syncthreads();
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t b = i < n_pairs ? lpt_bucket(read_off[i + 1] - read_off[i]) : 0u;
    if (i < n_pairs) atomicAdd(&lh[b], 1u);
    __syncthreads();
    for (int t = threadIdx.x; t < kLptBuckets; t += blockDim.x) {
        lpos[t] = lh[t] ? atomicAdd(&pos[t], lh[t]) : 0u;
        lh[t] = 0u;
    }
    __syncthreads();
    if (i < n_pairs) order[lpos[b] + atomicAdd(&lh[b], 1u)] = (uint32_t)i;
}

__global__ void k_zero_u32(uint32_t* p, uint32_t n) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

// Debug builds: the queue audit (batched form: a pair whose search hit is
// taken by exactly one window worker, a pair that ended in the search by
// none) and the hand-over of every audit bit to the pair's result flags.
__global__ void k_audit(AlignParams P, int queued) {
    const uint64_t pair = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (pair >= P.n_pairs || !P.audit) return;
    uint32_t a = P.audit[pair];
    if (queued) {
        const uint32_t expected = P.search[pair].row >= 0 ? 1u : 0u;
        if (a / kAuditTake != expected) a |= kAuditQueue;
    }
    if (a % kAuditTake) P.out[pair].flags |= GENASM_FLAG_INTERNAL;
    P.audit[pair] = a;
}

// Copies each pair's CIGAR elements to dst + dst_off[pair] (one block per pair).
__global__ void k_compact(const genasm_result* out, const uint64_t* dst_off, uint64_t n_pairs,
                          const uint32_t* cigar, uint32_t* dst) {
    const uint64_t pair = blockIdx.x;
    if (pair >= n_pairs) return;
    const genasm_result r = out[pair];
    for (uint32_t e = threadIdx.x; e < r.cigar_len; e += blockDim.x)
        dst[dst_off[pair] + e] = cigar[r.cigar_off + e];
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------

// The plain and unimproved kernels run the start search in their group's LDS first.
int plain_lds_bytes(int stride) {
    const int w = window_group_words(64, stride);
    return (w > kSearchGroupWords ? w : kSearchGroupWords) * 8;
}
int window_lds_bytes(int lds_rows, int stride) {
    const int easy = 4 * window_group_words(lds_rows, stride);
    const int hard = window_group_words(64, stride);
    return (easy > hard ? easy : hard) * 8;
}
int search_lds_bytes(int group_lanes) { return (64 / group_lanes) * kSearchGroupWords * 8; }

hipError_t launch_plain(const AlignParams& p, hipStream_t s) {
    if (p.n_pairs == 0) return hipSuccess;
    const int lds = plain_lds_bytes(p.stride);
    hipLaunchKernelGGL(k_plain, dim3((unsigned)p.n_pairs), dim3(64), lds, s, p);
    return hipGetLastError();
}

uint64_t unimproved_table_words(uint64_t n_pairs) { return n_pairs * kUnimpWords; }

hipError_t launch_unimproved(const AlignParams& p, unsigned long long* table, hipStream_t s) {
    if (p.n_pairs == 0) return hipSuccess;
    const int lds = plain_lds_bytes(p.stride);
    hipLaunchKernelGGL(k_unimproved, dim3((unsigned)p.n_pairs), dim3(64), lds, s, p, table);
    return hipGetLastError();
}

int search_blocks_per_cu(int group_lanes, int rows_per_lane) {
    int n = 0;
    const int lds = search_lds_bytes(group_lanes);
    hipError_t e = hipErrorInvalidValue;
    if (group_lanes == 64) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_search<64, 1>, 64, lds);
    else if (rows_per_lane == 1) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_search<16, 1>, 64, lds);
    else if (rows_per_lane == 2) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_search<16, 2>, 64, lds);
    else if (rows_per_lane == 4) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_search<16, 4>, 64, lds);
    return e == hipSuccess ? n : 0;
}

hipError_t launch_search(const AlignParams& p, int group_lanes, int rows_per_lane, int blocks,
                         hipStream_t s) {
    const int lds = search_lds_bytes(group_lanes);
    if (group_lanes == 64) {
        hipLaunchKernelGGL((k_search<64, 1>), dim3(blocks), dim3(64), lds, s, p);
    } else if (group_lanes == 16) {
        if (rows_per_lane == 1) hipLaunchKernelGGL((k_search<16, 1>), dim3(blocks), dim3(64), lds, s, p);
        else if (rows_per_lane == 2) hipLaunchKernelGGL((k_search<16, 2>), dim3(blocks), dim3(64), lds, s, p);
        else if (rows_per_lane == 4) hipLaunchKernelGGL((k_search<16, 4>), dim3(blocks), dim3(64), lds, s, p);
        else return hipErrorInvalidValue;
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_search_items(const AlignParams& p, uint32_t max_pairs, hipStream_t s) {
    if (max_pairs == 0) return hipSuccess;
    hipLaunchKernelGGL(k_search_items, dim3((max_pairs + 255) / 256), dim3(256), 0, s, p);
    return hipGetLastError();
}

hipError_t launch_search_finalize(const AlignParams& p, uint32_t max_pairs, hipStream_t s) {
    if (max_pairs == 0) return hipSuccess;
    hipLaunchKernelGGL(k_search_finalize, dim3((max_pairs + 255) / 256), dim3(256), 0, s, p);
    return hipGetLastError();
}

int compact_lds_bytes(int stride) { return 4 * compact_group_words(stride) * 8; }

int windows_blocks_per_cu(const AlignParams& p) {
    int n = 0;
    hipError_t e;
    if (p.compact)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_windows_c<false>, 64,
                                                         compact_lds_bytes(p.stride));
    else
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &n, p.hard_lanes == 64 ? k_windows<64> : p.hard_lanes == 32 ? k_windows<32> : k_windows<16>,
            64, window_lds_bytes(p.lds_rows, p.stride));
    return e == hipSuccess ? n : 0;
}

hipError_t launch_audit(const AlignParams& p, int queued, hipStream_t s) {
    if (!p.audit || p.n_pairs == 0) return hipSuccess;
    const unsigned blocks = (unsigned)((p.n_pairs + 255) / 256);
    hipLaunchKernelGGL(k_audit, dim3(blocks), dim3(256), 0, s, p, queued);
    return hipGetLastError();
}

hipError_t launch_windows(const AlignParams& p, int blocks, hipStream_t s) {
    if (p.compact) {
        const int lds = compact_lds_bytes(p.stride);
        if (p.stats) hipLaunchKernelGGL(k_windows_c<true>, dim3(blocks), dim3(64), lds, s, p);
        else hipLaunchKernelGGL(k_windows_c<false>, dim3(blocks), dim3(64), lds, s, p);
        return hipGetLastError();
    }
    const int lds = window_lds_bytes(p.lds_rows, p.stride);
    if (p.hard_lanes == 64) hipLaunchKernelGGL(k_windows<64>, dim3(blocks), dim3(64), lds, s, p);
    else if (p.hard_lanes == 32) hipLaunchKernelGGL(k_windows<32>, dim3(blocks), dim3(64), lds, s, p);
    else hipLaunchKernelGGL(k_windows<16>, dim3(blocks), dim3(64), lds, s, p);
    return hipGetLastError();
}

hipError_t launch_pack(const char* ascii, uint64_t n, uint8_t* packed, uint32_t* bad,
                       hipStream_t s) {
    const uint64_t bytes = (n + 3) / 4;
    if (bytes == 0) return hipSuccess;
    if (((uintptr_t)ascii & 15) == 0 && ((uintptr_t)packed & 3) == 0) {
        const uint64_t chunks = (n + 15) / 16;
        const unsigned blocks = (unsigned)((chunks + 255) / 256);
        hipLaunchKernelGGL(k_pack16, dim3(blocks), dim3(256), 0, s, ascii, n, packed, bad);
        return hipGetLastError();
    }
    const unsigned blocks = (unsigned)((bytes + 255) / 256);
    hipLaunchKernelGGL(k_pack, dim3(blocks), dim3(256), 0, s, ascii, n, packed, bad);
    return hipGetLastError();
}

hipError_t launch_init_counters(uint32_t* counters, uint32_t stage0_len, hipStream_t s) {
    hipLaunchKernelGGL(k_init_counters, dim3(1), dim3(64), 0, s, counters, stage0_len);
    return hipGetLastError();
}

hipError_t launch_serve_begin(uint32_t* cur, uint32_t* next, uint32_t* fin_len,
                              const uint32_t* params, const ServeAdmit* admit, ServeSlots slots,
                              uint32_t* new_list, hipStream_t s) {
    hipLaunchKernelGGL(k_serve_begin, dim3(1), dim3(256), 0, s, cur, next, fin_len, params, admit,
                       slots, new_list);
    return hipGetLastError();
}

hipError_t launch_serve_stamp(const uint32_t* params, TurnLimits* turn, hipStream_t s) {
    hipLaunchKernelGGL(k_serve_stamp, dim3(1), dim3(1), 0, s, params, turn);
    return hipGetLastError();
}

hipError_t launch_serve_finish(const uint32_t* fin_list, const uint32_t* fin_len,
                               const genasm_result* out, uint64_t* fin_off,
                               unsigned long long* hdr, uint32_t* sum_slot,
                               genasm_result* sum_res, const uint32_t* cigar, uint32_t* dst,
                               uint64_t dst_cap, uint32_t max_fin, hipStream_t s) {
    hipLaunchKernelGGL(k_serve_scan, dim3(1), dim3(1024), 0, s, fin_list, fin_len, out, fin_off,
                       hdr, sum_slot, sum_res, max_fin);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_serve_gather, dim3(1024), dim3(256), 0, s, fin_list, fin_len, out, fin_off,
                       cigar, dst, dst_cap, max_fin);
    return hipGetLastError();
}

hipError_t launch_scatter_bytes(const uint8_t* src, const uint64_t* src_off, uint8_t* dst,
                                const uint64_t* dst_off, const uint32_t* len, uint32_t n,
                                hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_scatter_bytes, dim3(n), dim3(256), 0, s, src, src_off, dst, dst_off, len, n);
    return hipGetLastError();
}

hipError_t launch_planes(const uint8_t* packed, const uint64_t* d_first, uint64_t n_bases,
                         unsigned long long* lo, unsigned long long* hi, hipStream_t s) {
    const uint64_t nwords = plane_words(n_bases);
    hipLaunchKernelGGL(k_planes, dim3((unsigned)((nwords + 255) / 256)), dim3(256), 0, s, packed,
                       d_first, n_bases, lo, hi, nwords);
    return hipGetLastError();
}

hipError_t launch_scatter_planes(const uint8_t* src, const uint64_t* src_off, const uint32_t* len,
                                 unsigned long long* lo, unsigned long long* hi,
                                 const uint64_t* dst_word, uint32_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_scatter_planes, dim3(n), dim3(256), 0, s, src, src_off, len, lo, hi,
                       dst_word, n);
    return hipGetLastError();
}

hipError_t launch_fill_u64(unsigned long long* p, uint64_t n, unsigned long long v, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_zero_u32(uint32_t* p, uint64_t n, hipStream_t s) {
    for (uint64_t at = 0; at < n; at += 1ull << 30) {
        const uint32_t k = (uint32_t)(n - at < (1ull << 30) ? n - at : (1ull << 30));
        hipLaunchKernelGGL(k_zero_u32, dim3((k + 255) / 256), dim3(256), 0, s, p + at, k);
    }
    return hipGetLastError();
}

hipError_t launch_lpt_order(const uint64_t* read_off, uint64_t n_pairs, uint32_t* hist,
                            uint32_t* order, hipStream_t s) {
    if (n_pairs == 0) return hipSuccess;
    const unsigned blocks = (unsigned)((n_pairs + 255) / 256);
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(kLptBuckets), 0, s, hist, (uint32_t)kLptBuckets);
    hipLaunchKernelGGL(k_lpt_count, dim3(blocks), dim3(256), kLptBuckets * 4, s, read_off, n_pairs, hist);
    hipLaunchKernelGGL(k_lpt_scan, dim3(1), dim3(kLptBuckets), 0, s, hist);
    hipLaunchKernelGGL(k_lpt_place, dim3(blocks), dim3(256), 2 * kLptBuckets * 4, s, read_off, n_pairs,
                       hist, order);
    return hipGetLastError();
}

hipError_t launch_compact_cigar(const genasm_result* d_out, const uint64_t* dst_off,
                                uint64_t n_pairs, const uint32_t* cigar, uint32_t* dst,
                                hipStream_t s) {
    if (n_pairs == 0) return hipSuccess;
    hipLaunchKernelGGL(k_compact, dim3((unsigned)n_pairs), dim3(64), 0, s, d_out, dst_off, n_pairs,
                       cigar, dst);
    return hipGetLastError();
}

}  // namespace genasm
