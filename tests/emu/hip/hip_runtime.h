// CPU emulation of the small HIP device surface the GenASM kernels use, so the
// unmodified kernel source builds with g++ for host-side debugging and tests.
//
// A launch runs its blocks one after another; each block runs its lanes as
// std::threads. Cross-lane operations (DPP moves, ballots, wave barriers) are
// emulated with a barrier per lane group: the kernels only ever exchange data
// inside a group of emu::group_lanes lanes, and every such operation is
// reached by all lanes of the group together. LDS is one global array; the
// part past a block's dynamic size is filled with a canary that is checked
// after the block.
#pragma once

#include <algorithm>
#include <atomic>
#include <barrier>
#include <cstddef>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <thread>
#include <vector>

#define __global__
#define __device__
#define __host__
#define __forceinline__ inline
#define __launch_bounds__(...)
#define __shared__

struct dim3 {
    unsigned x, y, z;
    dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};
struct alignas(16) uint4 {
    unsigned x, y, z, w;
};
typedef int hipError_t;
enum { hipSuccess = 0, hipErrorInvalidValue = 1 };
typedef struct ihipStream_t* hipStream_t;
typedef struct ihipEvent_t* hipEvent_t;
inline hipError_t hipGetLastError() { return hipSuccess; }
template <class K>
inline hipError_t hipOccupancyMaxActiveBlocksPerMultiprocessor(int* n, K, int, size_t) {
    *n = 1;
    return hipSuccess;
}

template <class A, class B>
inline auto min(A a, B b) -> decltype(a < b ? a : b) { return a < b ? a : b; }
template <class A, class B>
inline auto max(A a, B b) -> decltype(a < b ? a : b) { return a < b ? b : a; }

namespace emu {

struct BlockState {
    int lanes;
    int group_lanes;
    std::vector<std::unique_ptr<std::barrier<>>> bars;
    unsigned long long slot[256];
    bool pred[256];
};

struct LaneId {
    unsigned tid = 0, bid = 0, bdim = 64, gdim = 1;
    BlockState* blk = nullptr;
};

inline thread_local LaneId cur;
inline int group_lanes = 64;      // set by the driver before a launch
inline size_t lds_limit_bytes = 0;  // dynamic LDS of the current launch

inline dim3 thread_idx() { return dim3(cur.tid); }
inline dim3 block_idx() { return dim3(cur.bid); }
inline dim3 block_dim() { return dim3(cur.bdim); }
inline dim3 grid_dim() { return dim3(cur.gdim); }

inline void group_barrier() {
    cur.blk->bars[cur.tid / cur.blk->group_lanes]->arrive_and_wait();
}

inline int dpp_source(int lane, int ctrl) {
    switch (ctrl) {
        case 0x111: return (lane & 15) == 0 ? -1 : lane - 1;                  // row_shr:1
        case 0x121: return (lane & ~15) | ((lane - 1) & 15);                  // row_ror:1
        case 0x138: return lane == 0 ? -1 : lane - 1;                         // wave_shr:1
        case 0x13C: return (lane + 63) & 63;                                  // wave_ror:1
        default:
            std::fprintf(stderr, "emu: unsupported DPP control %#x\n", ctrl);
            std::abort();
    }
}

inline int update_dpp(int old, int src, int ctrl, int row_mask, int bank_mask, bool bound_ctrl) {
    (void)row_mask; (void)bank_mask;
    BlockState* b = cur.blk;
    const int lane = (int)cur.tid;
    b->slot[lane] = (unsigned)src;
    group_barrier();
    const int from = dpp_source(lane, ctrl);
    int out;
    if (from < 0) out = bound_ctrl ? 0 : old;
    else {
        if (from / b->group_lanes != lane / b->group_lanes) {
            // 32-lane groups shift with wave_shr:1 and replace what lane 32 reads
            // from lane 31; a poison value stands in for it
            if (!(ctrl == 0x138 && b->group_lanes == 32)) {
                std::fprintf(stderr, "emu: DPP read across lane groups (%d <- %d)\n", lane, from);
                std::abort();
            }
            out = (int)0x5EED5EEDu;
        } else {
            out = (int)(unsigned)b->slot[from];
        }
    }
    group_barrier();
    return out;
}

inline unsigned long long ballot(bool p) {
    BlockState* b = cur.blk;
    const int lane = (int)cur.tid;
    b->pred[lane] = p;
    group_barrier();
    unsigned long long m = 0;
    const int g0 = lane / b->group_lanes * b->group_lanes;
    for (int l = g0; l < g0 + b->group_lanes; ++l)
        if (b->pred[l]) m |= 1ull << (l & 63);
    group_barrier();
    return m;
}

// Value of `v` in lane `src` of the calling lane's group.
template <class T>
inline T shfl(T v, int src) {
    BlockState* b = cur.blk;
    const int lane = (int)cur.tid;
    group_barrier();
    b->slot[lane] = (unsigned long long)v;
    group_barrier();
    const int g0 = lane / b->group_lanes * b->group_lanes;
    const T out = (T)b->slot[g0 + (src % b->group_lanes)];
    group_barrier();
    return out;
}

constexpr unsigned long long kCanary = 0xC0FFEE11DEADBEEFull;

template <class K, class... Args>
void launch(K kernel, dim3 grid, dim3 block, size_t lds_bytes, unsigned long long* lds,
            size_t lds_words, Args... args) {
    if (block.x > 256 || lds_bytes > lds_words * 8) {
        std::fprintf(stderr, "emu: launch shape not supported (block %u, lds %zu)\n", block.x, lds_bytes);
        std::abort();
    }
    for (unsigned bid = 0; bid < grid.x; ++bid) {
        for (size_t w = 0; w < lds_words; ++w) lds[w] = w * 8 < lds_bytes ? 0xABABABABABABABABull : kCanary;
        BlockState bs;
        bs.lanes = (int)block.x;
        bs.group_lanes = std::min<int>(group_lanes, (int)block.x);
        for (int g = 0; g < bs.lanes / bs.group_lanes; ++g)
            bs.bars.emplace_back(new std::barrier<>(bs.group_lanes));
        std::vector<std::thread> th;
        for (unsigned t = 0; t < block.x; ++t) {
            th.emplace_back([&, t]() {
                cur.tid = t;
                cur.bid = bid;
                cur.bdim = block.x;
                cur.gdim = grid.x;
                cur.blk = &bs;
                kernel(args...);
            });
        }
        for (auto& x : th) x.join();
        for (size_t w = (lds_bytes + 7) / 8; w < lds_words; ++w) {
            if (lds[w] != kCanary) {
                std::fprintf(stderr, "emu: LDS write past the dynamic size at word %zu\n", w);
                std::abort();
            }
        }
    }
}

}  // namespace emu

#define threadIdx (emu::thread_idx())
#define blockIdx (emu::block_idx())
#define blockDim (emu::block_dim())
#define gridDim (emu::grid_dim())

namespace emu {
inline unsigned long long bitreverse64(unsigned long long x) {
    unsigned long long r = 0;
    for (int b = 0; b < 64; ++b) r |= ((x >> b) & 1ull) << (63 - b);
    return r;
}
}  // namespace emu
#define __builtin_bitreverse64 emu::bitreverse64
inline unsigned long long clock64() { return 0ull; }
namespace emu {
inline std::atomic<unsigned long long> clock_reads{0};
}  // namespace emu
// The device clock, read by a scalar instruction on the GPU (one value per
// wavefront): here one value per lane group, advancing by one per read.
inline unsigned long long wall_clock64() {
    emu::BlockState* b = emu::cur.blk;
    const int lane = (int)emu::cur.tid;
    const int g0 = lane / b->group_lanes * b->group_lanes;
    emu::group_barrier();
    if (lane == g0) b->slot[lane] = emu::clock_reads.fetch_add(1);
    emu::group_barrier();
    const unsigned long long v = b->slot[g0];
    emu::group_barrier();
    return v;
}
inline void __threadfence_system() { std::atomic_thread_fence(std::memory_order_seq_cst); }
namespace emu {
// The first lane's value to every lane: here the first lane of the group.
inline int readfirstlane(int v) {
    BlockState* b = cur.blk;
    const int lane = (int)cur.tid;
    const int g0 = lane / b->group_lanes * b->group_lanes;
    group_barrier();
    if (lane == g0) b->slot[lane] = (unsigned long long)(unsigned)v;
    group_barrier();
    const int r = (int)(unsigned)b->slot[g0];
    group_barrier();
    return r;
}
}  // namespace emu
#define __builtin_amdgcn_readfirstlane emu::readfirstlane
#define __builtin_amdgcn_update_dpp emu::update_dpp
namespace emu {
inline int mov_dpp(int src, int ctrl, int row_mask, int bank_mask, bool bound_ctrl) {
    // lanes without a source lane would keep an undefined value; the kernels
    // use this only for rotations, where every lane has one
    return update_dpp((int)0xDEADDEAD, src, ctrl, row_mask, bank_mask, bound_ctrl);
}
}  // namespace emu
#define __builtin_amdgcn_mov_dpp emu::mov_dpp
namespace emu {
// v_alignbit_b32: the low 32 bits of (hi:lo) >> (s mod 32)
inline unsigned alignbit(unsigned hi, unsigned lo, unsigned s) {
    return (unsigned)((((unsigned long long)hi << 32) | lo) >> (s & 31));
}
}  // namespace emu
#define __builtin_amdgcn_alignbit emu::alignbit
// Block-wide barriers and static shared arrays are not emulated (kernels that
// use them, such as the ordering scan, do not run under the emulation).
inline void __syncthreads() {
    std::fprintf(stderr, "emu: __syncthreads is not emulated\n");
    std::abort();
}
#define __builtin_amdgcn_s_waitcnt(x) emu::group_barrier()
#define __builtin_amdgcn_wave_barrier() emu::group_barrier()
#define __builtin_amdgcn_fence(order, scope) std::atomic_thread_fence(std::memory_order_seq_cst)
#define __ballot(p) emu::ballot(p)
#define __shfl(v, src) emu::shfl(v, src)
#define __HIP_MEMORY_SCOPE_AGENT 0
#define __HIP_MEMORY_SCOPE_SYSTEM 0
#define __HIP_MEMORY_SCOPE_WAVEFRONT 0
#define __hip_atomic_load(p, order, scope) __atomic_load_n((p), __ATOMIC_SEQ_CST)

template <class T>
inline T atomicAdd(T* p, T v) { return __atomic_fetch_add(p, v, __ATOMIC_SEQ_CST); }
template <class T>
inline T atomicOr(T* p, T v) { return __atomic_fetch_or(p, v, __ATOMIC_SEQ_CST); }
template <class T>
inline T atomicMin(T* p, T v) {
    T cur = __atomic_load_n(p, __ATOMIC_SEQ_CST);
    while (v < cur && !__atomic_compare_exchange_n(p, &cur, v, false, __ATOMIC_SEQ_CST,
                                                   __ATOMIC_SEQ_CST)) {
    }
    return cur;
}

namespace genasm { extern unsigned long long smem[]; }
constexpr size_t kEmuLdsWords = 160 * 1024 / 8;
#define hipLaunchKernelGGL(kernel, grid, block, lds, stream, ...) \
    emu::launch(kernel, grid, block, lds, genasm::smem, kEmuLdsWords, __VA_ARGS__)
