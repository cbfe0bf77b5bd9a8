// Microbenchmarks of the gfx950 limits the window kernel is measured
// against: the rate of the DC recurrence's own integer instruction mix in
// registers, plain 32-bit integer VALU throughput, the issue rates of the
// instruction kinds the recurrence is built from (64-bit shift, 32-bit funnel
// shift, DPP lane move), LDS bandwidth and HBM bandwidth. Each kernel's work is
// known exactly, so achieved rate = work / time of the launch (HIP events).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cstring>

#include "internal.h"

namespace {

typedef unsigned long long u64;

constexpr int kChains = 8;        // independent recurrence chains per lane
constexpr int kMixSteps = 4096;   // steps of each chain per launch

// The DC step, as the window kernels execute it, on kChains independent
// chains: one DPP lane shift of a 64-bit word (the row above), then
//   x = D & (((D & up) << 1) | low);  R = x & ((R << 1) | pm)
// on 32-bit halves (the high halves' shifts as funnel shifts), counted as its
// 6 64-bit operations = 12 int32 lane-operations per step and chain. The
// result is stored so that nothing is optimized away.
__global__ __launch_bounds__(256) void k_peak_mix(const u64* in, u64* out) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    u64 R[kChains], D[kChains];
    const u64 pm0 = in[0] ^ (u64)t, low = in[1] & 1ull;
#pragma unroll
    for (int c = 0; c < kChains; ++c) {
        R[c] = in[2 + c] + (u64)t;
        D[c] = in[2 + kChains + c] ^ (u64)t;
    }
    for (int s = 0; s < kMixSteps; ++s) {
        const u64 pm = pm0 + (u64)s;  // one addition per step for all chains
#pragma unroll
        for (int c = 0; c < kChains; ++c) {
            const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp((int)(unsigned)R[c],
                                                                      (int)(unsigned)R[c], 0x111,
                                                                      0xF, 0xF, false);
            const unsigned hi = (unsigned)__builtin_amdgcn_update_dpp(
                (int)(unsigned)(R[c] >> 32), (int)(unsigned)(R[c] >> 32), 0x111, 0xF, 0xF, false);
            const u64 up = ((u64)hi << 32) | lo;
            const uint32_t Rl = (uint32_t)R[c], Rh = (uint32_t)(R[c] >> 32);
            const uint32_t Dl = (uint32_t)D[c], Dh = (uint32_t)(D[c] >> 32);
            const uint32_t el = Dl & lo, eh = Dh & hi;
            const uint32_t xl = Dl & ((el << 1) | (uint32_t)low);
            const uint32_t xh = Dh & __builtin_amdgcn_alignbit(eh, el, 31);
            const uint32_t sl = (Rl << 1) | (uint32_t)pm;
            const uint32_t sh = __builtin_amdgcn_alignbit(Rh, Rl, 31) | (uint32_t)(pm >> 32);
            D[c] = up;
            R[c] = ((u64)(xh & sh) << 32) | (xl & sl);
        }
    }
    u64 acc = 0;
#pragma unroll
    for (int c = 0; c < kChains; ++c) acc ^= R[c] ^ D[c];
    out[t] = acc;
}

// Plain 32-bit integer VALU throughput: kChains independent chains of
// and/or/xor (3 int32 lane-operations per step and chain).
__global__ __launch_bounds__(256) void k_peak_int32(const unsigned* in, unsigned* out) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    unsigned a[kChains];
    const unsigned b = in[0] ^ (unsigned)t, c2 = in[1] | (unsigned)t;
#pragma unroll
    for (int c = 0; c < kChains; ++c) a[c] = in[2 + c] + (unsigned)t;
    for (int s = 0; s < kMixSteps; ++s) {
#pragma unroll
        for (int c = 0; c < kChains; ++c) a[c] = ((a[c] & b) | c2) ^ (unsigned)s;
    }
    unsigned acc = 0;
#pragma unroll
    for (int c = 0; c < kChains; ++c) acc ^= a[c];
    out[t] = acc;
}

// Issue rate of one instruction kind: kChains independent chains per lane,
// each instruction reading and writing its own chain. OP 0: v_lshlrev_b64 by
// one; OP 1: v_alignbit_b32 (32-bit funnel shift); OP 2: v_mov_b32_dpp row
// rotation by one lane.
template <int OP>
__device__ __forceinline__ void op_step(u64& a) {
#if defined(__HIP_DEVICE_COMPILE__)
    if constexpr (OP == 0) {
        asm volatile("v_lshlrev_b64 %0, 1, %0" : "+v"(a));
    } else {
        uint32_t lo = (uint32_t)a;
        const uint32_t hi = (uint32_t)(a >> 32);
        if constexpr (OP == 1) asm volatile("v_alignbit_b32 %0, %0, %1, 31" : "+v"(lo) : "v"(hi));
        else asm volatile("v_mov_b32_dpp %0, %0 row_ror:1 row_mask:0xf bank_mask:0xf" : "+v"(lo));
        a = ((u64)hi << 32) | lo;
    }
#else
    a = a << 1;
#endif
}
template <int OP>
__global__ __launch_bounds__(256) void k_peak_op(const u64* in, u64* out) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    u64 a[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) a[c] = in[2 + c] ^ (u64)t;
    for (int s = 0; s < kMixSteps; ++s) {
#pragma unroll
        for (int c = 0; c < kChains; ++c) op_step<OP>(a[c]);
    }
    u64 acc = 0;
#pragma unroll
    for (int c = 0; c < kChains; ++c) acc ^= a[c];
    out[t] = acc;
}

// LDS bandwidth: every lane reads 16 bytes per step from a 32 KB block
// (consecutive lanes consecutive 16-byte words: no bank conflicts).
constexpr int kLdsSteps = 2048;
constexpr int kLdsWords = 2048;  // uint4 words per block (32 KB)
__global__ __launch_bounds__(256) void k_peak_lds(const unsigned* in, unsigned* out) {
    __shared__ uint4 buf[kLdsWords];
    const int t = threadIdx.x;
    for (int w = t; w < kLdsWords; w += blockDim.x)
        buf[w] = make_uint4(in[0] + w, in[1] ^ w, w, ~w);
    __syncthreads();
    // the index step comes from memory (256 at run time), so the compiler
    // cannot see that the reads repeat and keep them in registers
    const int inc = 256 + (int)((in[3] & 1u) << 8);
    unsigned acc = 0;
    int idx = t;
    for (int s = 0; s < kLdsSteps; ++s) {
        const uint4 v = buf[idx];
        acc ^= v.x ^ v.y ^ v.z ^ v.w;
        idx = (idx + inc) & (kLdsWords - 1);
    }
    out[blockIdx.x * blockDim.x + t] = acc;
}

// HBM bandwidth: a streaming copy of n 16-byte words (each read once and
// written once), grid-stride.
__global__ __launch_bounds__(256) void k_peak_copy(const uint4* src, uint4* dst, uint64_t n) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

}  // namespace

extern "C" {

int genasm_measure_peaks(genasm_ctx* ctx, genasm_peaks* out) {
    if (!ctx || !out) return GENASM_E_INVAL;
    std::memset(out, 0, sizeof(*out));
    if (hipSetDevice(ctx->device) != hipSuccess) return GENASM_E_DEVICE;
    hipStream_t s = ctx->stream;
    const int cus = ctx->num_cus;
    // enough 256-thread blocks for full occupancy on every CU, several times over
    const int blocks = cus * 32;
    const int threads = blocks * 256;
    const uint64_t copy_words = 1ull << 26;  // 1 GiB read, 1 GiB written
    u64 *d_in = nullptr, *d_out = nullptr;
    uint4 *d_src = nullptr, *d_dst = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = GENASM_OK;
    auto timed = [&](auto launch, float* ms) -> bool {
        launch();  // warm-up
        if (hipEventRecord(e0, s) != hipSuccess) return false;
        launch();
        if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) return false;
        return hipEventElapsedTime(ms, e0, e1) == hipSuccess && hipGetLastError() == hipSuccess;
    };
    do {
        if (hipMalloc(&d_in, 64 * sizeof(u64)) != hipSuccess ||
            hipMalloc(&d_out, (size_t)threads * sizeof(u64)) != hipSuccess ||
            hipMalloc(&d_src, copy_words * sizeof(uint4)) != hipSuccess ||
            hipMalloc(&d_dst, copy_words * sizeof(uint4)) != hipSuccess) {
            rc = GENASM_E_NOMEM;
            break;
        }
        if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess ||
            hipMemsetAsync(d_in, 0x5A, 64 * sizeof(u64), s) != hipSuccess ||
            hipMemsetAsync(d_src, 0x11, copy_words * sizeof(uint4), s) != hipSuccess) {
            rc = GENASM_E_DEVICE;
            break;
        }
        float ms = 0.f;
        if (!timed([&] { hipLaunchKernelGGL(k_peak_mix, dim3(blocks), dim3(256), 0, s, d_in, d_out); }, &ms)) {
            rc = GENASM_E_DEVICE;
            break;
        }
        out->dc_mix_tops = (double)threads * kMixSteps * kChains * 12 / (ms / 1e3) / 1e12;
        if (!timed([&] {
                hipLaunchKernelGGL(k_peak_int32, dim3(blocks), dim3(256), 0, s,
                                   reinterpret_cast<const unsigned*>(d_in), reinterpret_cast<unsigned*>(d_out));
            }, &ms)) {
            rc = GENASM_E_DEVICE;
            break;
        }
        out->int32_tops = (double)threads * kMixSteps * kChains * 3 / (ms / 1e3) / 1e12;
        if (!timed([&] {
                hipLaunchKernelGGL(k_peak_lds, dim3(blocks), dim3(256), 0, s,
                                   reinterpret_cast<const unsigned*>(d_in), reinterpret_cast<unsigned*>(d_out));
            }, &ms)) {
            rc = GENASM_E_DEVICE;
            break;
        }
        out->lds_tbps = (double)threads * kLdsSteps * 16 / (ms / 1e3) / 1e12;
        // a 64-bit shift counts as two int32 lane-operations, the others as one
        const double op_work = (double)threads * kMixSteps * kChains;
        double* const op_out[3] = {&out->shift64_tops, &out->funnel_tops, &out->dpp_tops};
        bool op_ok = true;
        for (int op = 0; op < 3 && op_ok; ++op) {
            op_ok = timed([&] {
                if (op == 0) hipLaunchKernelGGL(k_peak_op<0>, dim3(blocks), dim3(256), 0, s, d_in, d_out);
                else if (op == 1) hipLaunchKernelGGL(k_peak_op<1>, dim3(blocks), dim3(256), 0, s, d_in, d_out);
                else hipLaunchKernelGGL(k_peak_op<2>, dim3(blocks), dim3(256), 0, s, d_in, d_out);
            }, &ms);
            *op_out[op] = op_work * (op == 0 ? 2 : 1) / (ms / 1e3) / 1e12;
        }
        if (!op_ok) {
            rc = GENASM_E_DEVICE;
            break;
        }
        if (!timed([&] {
                hipLaunchKernelGGL(k_peak_copy, dim3(cus * 16), dim3(256), 0, s, d_src, d_dst, copy_words);
            }, &ms)) {
            rc = GENASM_E_DEVICE;
            break;
        }
        out->hbm_tbps = (double)copy_words * 16 * 2 / (ms / 1e3) / 1e12;
        out->compute_units = cus;
    } while (false);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    for (void* p : {(void*)d_in, (void*)d_out, (void*)d_src, (void*)d_dst})
        if (p) (void)hipFree(p);
    return rc;
}

}  // extern "C"
