// Host runtime of the GenASM library: context, argument checks, device
// scratch, launch orchestration for the plain and batched forms, and the
// host-memory convenience call.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "internal.h"
#include "trace.h"

using namespace genasm;

// Device scratch of genasm_batch_align_dev_noalloc, one copy on every GPU the
// library runs on, held until the process ends. In host code the name stands
// for a host-side shadow, not a device address: host code reaches the array
// only through the address static_scratch_ptr obtained for the device.
static __device__ __align__(256) char scratch[GENASM_NOALLOC_SCRATCH_BYTES];

namespace {

// Device address of `scratch` on each device, looked up once per device (with
// that device current) by genasm_create.
std::mutex g_static_mu;
constexpr int kMaxDevices = 64;
void* g_static_ptr[kMaxDevices] = {};

hipError_t static_scratch_ptr(int device, void** out) {
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_static_mu);
    if (!g_static_ptr[device]) {
        void* ptr = nullptr;
        hipError_t e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!ptr) return hipErrorInvalidSymbol;
        g_static_ptr[device] = ptr;
    }
    *out = g_static_ptr[device];
    return hipSuccess;
}


#define CHECK_HIP(ctx, expr)                                                              \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess) return set_err(ctx, GENASM_E_DEVICE, #expr, e_);            \
    } while (0)

int set_err(genasm_ctx* ctx, int code, const char* what, hipError_t e = hipSuccess) {
    if (ctx) {
        ctx->err = what ? what : "";
        if (e != hipSuccess) {
            ctx->err += ": ";
            ctx->err += hipGetErrorString(e);
        }
    }
    return code;
}

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Grows a device buffer to at least `need` bytes (contents are not kept).
// A pinned context (one whose buffers a captured graph may use) never frees or
// moves them: the call fails instead.
int ensure(genasm_ctx* ctx, char** buf, size_t* cap, size_t need) {
    if (need <= *cap) return GENASM_OK;
    if (ctx->pinned)
        return set_err(ctx, GENASM_E_PINNED,
                       "the context's device buffers are held by a captured graph and cannot grow: "
                       "size them with an eager call before capture, or call genasm_unpin once "
                       "no graph uses them");
    if (*buf) {
        // the buffer may be in use by earlier calls on any stream
        hipError_t e = hipDeviceSynchronize();
        if (e != hipSuccess) return set_err(ctx, GENASM_E_DEVICE, "hipDeviceSynchronize", e);
        (void)hipFree(*buf);
        *buf = nullptr;
        *cap = 0;
    }
    size_t want = align_up(std::max(need, (size_t)1 << 20), (size_t)1 << 20);
    // failure injection for tests of the error path: GENASM_FAIL_ALLOC=1 makes
    // every growth of a context buffer fail as if the device were full
    const char* fail = std::getenv("GENASM_FAIL_ALLOC");
    hipError_t e = fail && fail[0] == '1' ? hipErrorOutOfMemory : hipMalloc((void**)buf, want);
    if (e != hipSuccess) {
        *buf = nullptr;
        (void)hipGetLastError();
        return set_err(ctx, GENASM_E_NOMEM, "hipMalloc scratch", e);
    }
    *cap = want;
    return GENASM_OK;
}

// Characters of one CIGAR run as text ("12=").
inline uint64_t cigar_run_chars(uint32_t e) {
    uint32_t len = GENASM_CIGAR_LEN(e);
    uint64_t digits = 1;
    while (len >= 10) { len /= 10; ++digits; }
    return digits + 1;
}

// Writes one CIGAR run as text at w; returns the position after it.
inline char* cigar_run_text(uint32_t e, char* w) {
    static const char kOp[4] = {'=', 'X', 'I', 'D'};
    char tmp[12];
    int k = 0;
    uint32_t len = GENASM_CIGAR_LEN(e);
    do { tmp[k++] = (char)('0' + len % 10); len /= 10; } while (len);
    while (k) *w++ = tmp[--k];
    *w++ = kOp[GENASM_CIGAR_OP(e)];
    return w;
}

struct Carver {
    char* base;
    size_t off = 0;
    template <class T>
    T* take(size_t count) {
        off = align_up(off, 256);
        T* p = reinterpret_cast<T*>(base ? base + off : nullptr);
        off += count * sizeof(T);
        return p;
    }
};

bool valid_wko(int32_t k, int32_t W, int32_t O) {
    return W >= 2 && W <= 64 && O >= 0 && O < W && k >= 0;
}

// Workload signature of a batch for the tuning cache: powers of two of the
// pair count and of the mean read length, and k, W, O.
std::string tune_key(uint64_t n_pairs, uint64_t total_read_bases, int32_t k, int32_t W, int32_t O) {
    auto lg = [](uint64_t x) { int e = 0; while (x > 1) { x >>= 1; ++e; } return e; };
    const uint64_t mean = n_pairs ? total_read_bases / n_pairs : 0;
    return "n" + std::to_string(lg(n_pairs)) + "_m" + std::to_string(lg(mean)) + "_k" +
           std::to_string(std::min(k, W)) + "_W" + std::to_string(W) + "_O" + std::to_string(O);
}

int resolve_launch(const genasm_launch* in, genasm_launch* out) {
    genasm_default_launch(in ? in->form : GENASM_FORM_BATCHED, out);
    if (!in) return GENASM_OK;
    if (in->form != GENASM_FORM_PLAIN && in->form != GENASM_FORM_BATCHED &&
        in->form != GENASM_FORM_UNIMPROVED)
        return GENASM_E_INVAL;
    if (in->group_lanes) out->group_lanes = in->group_lanes;
    if (in->search_lanes) out->search_lanes = in->search_lanes;
    if (in->lds_rows) out->lds_rows = in->lds_rows;
    out->workers_per_cu = in->workers_per_cu;
    if (in->lpt_order >= 0) out->lpt_order = in->lpt_order;
    if (in->hard_row < -1) return GENASM_E_INVAL;
    if (in->hard_row) out->hard_row = in->hard_row < 0 ? 0 : in->hard_row;  // -1: every pair
    if (in->hard_lanes) out->hard_lanes = in->hard_lanes;
    if (in->tb_prefetch >= 0) out->tb_prefetch = in->tb_prefetch;
    if (out->tb_prefetch != 0 && out->tb_prefetch != 1) return GENASM_E_INVAL;
    if (in->hard_share >= 0) out->hard_share = in->hard_share;
    if (out->hard_share > 100) return GENASM_E_INVAL;
    if (in->table_bits) out->table_bits = in->table_bits;
    if (out->table_bits != 32 && out->table_bits != 64) return GENASM_E_INVAL;
    if (in->search_per_cu) out->search_per_cu = in->search_per_cu;
    if (out->search_per_cu < 1 || out->search_per_cu > 32) return GENASM_E_INVAL;
    if (out->hard_lanes != 16 && out->hard_lanes != 32 && out->hard_lanes != 64)
        return GENASM_E_INVAL;
    if (out->group_lanes != 16 && out->group_lanes != 64) return GENASM_E_INVAL;
    if (out->search_lanes != 16 && out->search_lanes != 64) return GENASM_E_INVAL;
    if (out->lds_rows < 16 || out->lds_rows > 64 || out->lds_rows % 16) return GENASM_E_INVAL;
    if (out->workers_per_cu < 0 || out->workers_per_cu > 32) return GENASM_E_INVAL;
    if (out->hard_row < 0 || out->hard_row > 65) return GENASM_E_INVAL;
    // 32-lane hard groups spill rows 32..63 into two 16-lane groups' spill areas
    if (out->hard_lanes == 32 && out->lds_rows > 48) return GENASM_E_INVAL;
    if (out->group_lanes == 64) {
        // every pair on the whole-wavefront path
        out->hard_row = 0;
        out->hard_lanes = 64;
    }
    return GENASM_OK;
}

}  // namespace

extern "C" {

const char* genasm_version(void) { return "genasm-gfx950 0.1"; }

const char* genasm_strerror(int code) {
    switch (code) {
        case GENASM_OK: return "ok";
        case GENASM_E_INVAL: return "invalid argument";
        case GENASM_E_ALPHABET: return "sequence byte outside ACGTacgt";
        case GENASM_E_NOMEM: return "out of memory";
        case GENASM_E_DEVICE: return "HIP device error";
        case GENASM_E_NOSPACE: return "output buffer too small";
        case GENASM_E_BUSY: return "request refused: admission budget exhausted";
        case GENASM_E_TOOLONG: return "sequence longer than 2^31-1 bases";
        case GENASM_E_PINNED: return "context buffers are held by a captured graph";
        case GENASM_E_SCRATCH: return "batch needs more than the no-allocation call's static scratch";
        default: return "unknown error";
    }
}

int genasm_default_launch(int32_t form, genasm_launch* out) {
    if (!out) return GENASM_E_INVAL;
    std::memset(out, 0, sizeof(*out));
    out->form = form;
    out->group_lanes = 16;
    out->search_lanes = 16;
    out->lds_rows = 16;
    out->workers_per_cu = 0;
    out->lpt_order = 1;
    out->hard_row = 16;
    out->hard_lanes = 16;
    out->tb_prefetch = 0;
    out->hard_share = 50;
    out->table_bits = 64;
    out->search_per_cu = 8;
    return GENASM_OK;
}

// Reason of the last genasm_create failure on this thread.
static thread_local std::string g_create_err;

static int create_fail(int code, const char* what, hipError_t e) {
    g_create_err = what;
    if (e != hipSuccess) {
        g_create_err += ": ";
        g_create_err += hipGetErrorString(e);
    }
    (void)hipGetLastError();
    return code;
}

int genasm_create(genasm_ctx** out, int hip_device) {
    if (!out) return GENASM_E_INVAL;
    *out = nullptr;
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess) return create_fail(GENASM_E_DEVICE, "hipGetDeviceCount", e);
    if (hip_device < 0 || hip_device >= count)
        return create_fail(GENASM_E_DEVICE, "no such HIP device", hipSuccess);
    int major = 0, minor = 0, cus = 0;
    if ((e = hipDeviceGetAttribute(&major, hipDeviceAttributeComputeCapabilityMajor, hip_device)) ||
        (e = hipDeviceGetAttribute(&minor, hipDeviceAttributeComputeCapabilityMinor, hip_device)) ||
        (e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, hip_device)))
        return create_fail(GENASM_E_DEVICE, "hipDeviceGetAttribute", e);
    if (major != 9 || minor != 5)  // the code objects are built for gfx950 only
        return create_fail(GENASM_E_DEVICE, "device is not gfx950", hipSuccess);
    genasm_ctx* ctx = new (std::nothrow) genasm_ctx();
    if (!ctx) return GENASM_E_NOMEM;
    ctx->device = hip_device;
    ctx->num_cus = cus;
    if ((e = hipSetDevice(hip_device)) != hipSuccess) {
        delete ctx;
        return create_fail(GENASM_E_DEVICE, "hipSetDevice", e);
    }
    if ((e = hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking)) != hipSuccess) {
        delete ctx;
        return create_fail(GENASM_E_DEVICE, "hipStreamCreateWithFlags", e);
    }
    // the no-allocation entry point's scratch on this device
    if ((e = static_scratch_ptr(hip_device, &ctx->static_scratch)) != hipSuccess) {
        (void)hipStreamDestroy(ctx->stream);
        delete ctx;
        return create_fail(GENASM_E_DEVICE, "hipGetSymbolAddress of the static scratch", e);
    }
    *out = ctx;
    return GENASM_OK;
}

void genasm_destroy(genasm_ctx* ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    if (ctx->scratch) (void)hipFree(ctx->scratch);
    if (ctx->planes) (void)hipFree(ctx->planes);
    if (ctx->unimp) (void)hipFree(ctx->unimp);
    if (ctx->stage) (void)hipFree(ctx->stage);
    if (ctx->dbg) (void)hipFree(ctx->dbg);
    if (ctx->stats) (void)hipFree(ctx->stats);
    for (hipEvent_t e : ctx->ev)
        if (e) (void)hipEventDestroy(e);
    if (ctx->stream) (void)hipStreamDestroy(ctx->stream);
    delete ctx;
}

int genasm_unpin(genasm_ctx* ctx) {
    if (!ctx) return GENASM_E_INVAL;
    ctx->pinned = false;
    return GENASM_OK;
}

const char* genasm_last_error(const genasm_ctx* ctx) {
    return ctx ? ctx->err.c_str() : g_create_err.c_str();
}

int genasm_pack(const char* ascii, uint64_t n, uint8_t* packed, uint64_t* bad_index) {
    if ((!ascii || !packed) && n) return GENASM_E_INVAL;
    for (uint64_t byte = 0; byte * 4 < n; ++byte) {
        unsigned v = 0;
        for (int u = 0; u < 4; ++u) {
            const uint64_t b = byte * 4 + u;
            if (b >= n) break;
            unsigned code;
            switch (ascii[b]) {
                case 'A': case 'a': code = 0; break;
                case 'C': case 'c': code = 1; break;
                case 'G': case 'g': code = 2; break;
                case 'T': case 't': code = 3; break;
                default:
                    if (bad_index) *bad_index = b;
                    return GENASM_E_ALPHABET;
            }
            v |= code << (2 * u);
        }
        packed[byte] = (uint8_t)v;
    }
    return GENASM_OK;
}

static int check_offsets(const uint64_t* off, uint64_t n_pairs, uint64_t stream_len) {
    for (uint64_t i = 0; i < n_pairs; ++i) {
        if (off[i + 1] < off[i]) return GENASM_E_INVAL;
        if (off[i + 1] - off[i] > 0x7fffffffull) return GENASM_E_TOOLONG;
    }
    if (stream_len != UINT64_MAX && off[n_pairs] > stream_len) return GENASM_E_INVAL;
    return GENASM_OK;
}

static bool ascii_ok(unsigned char c) {
    switch (c) {
        case 'A': case 'C': case 'G': case 'T': case 'a': case 'c': case 'g': case 't': return true;
        default: return false;
    }
}

int genasm_validate(const char* reads, uint64_t reads_len, const uint64_t* read_off,
                    const char* refs, uint64_t refs_len, const uint64_t* ref_off,
                    uint64_t n_pairs, int32_t k, int32_t W, int32_t O) {
    if (!valid_wko(k, W, O)) return GENASM_E_INVAL;
    if (!read_off || !ref_off) return GENASM_E_INVAL;
    int rc = check_offsets(read_off, n_pairs, reads_len);
    if (rc) return rc;
    rc = check_offsets(ref_off, n_pairs, refs_len);
    if (rc) return rc;
    if ((!reads && read_off[n_pairs] > read_off[0]) || (!refs && ref_off[n_pairs] > ref_off[0]))
        return GENASM_E_INVAL;
    for (uint64_t b = read_off[0]; b < read_off[n_pairs]; ++b)
        if (!ascii_ok((unsigned char)reads[b])) return GENASM_E_ALPHABET;
    for (uint64_t b = ref_off[0]; b < ref_off[n_pairs]; ++b)
        if (!ascii_ok((unsigned char)refs[b])) return GENASM_E_ALPHABET;
    return GENASM_OK;
}

int genasm_pack_dev(genasm_ctx* ctx, const char* d_ascii, uint64_t n, uint8_t* d_packed,
                    uint32_t* d_bad_count, void* stream) {
    if (!ctx) return GENASM_E_INVAL;
    if (n && (!d_ascii || !d_packed || !d_bad_count)) return set_err(ctx, GENASM_E_INVAL, "null pointer");
    hipStream_t s = (hipStream_t)stream;  // NULL: the null stream
    CHECK_HIP(ctx, hipSetDevice(ctx->device));
    CHECK_HIP(ctx, launch_pack(d_ascii, n, d_packed, d_bad_count, s));
    return GENASM_OK;
}

}  // extern "C"

namespace {

// The device-form call. Scratch (bit planes, search lists, queues, table
// spill, profiling counters) comes from the context's buffers, grown on
// demand, or with `noalloc` from the static `scratch` array, in which case
// nothing is allocated and profiling is not recorded.
int align_dev(genasm_ctx* ctx, const uint8_t* d_reads2b, const uint64_t* d_read_off,
              const uint8_t* d_refs2b, const uint64_t* d_ref_off, uint64_t n_pairs,
              uint64_t total_read_bases, uint64_t total_ref_bases, int32_t k, int32_t W, int32_t O,
              genasm_result* d_out, uint32_t* d_cigar, uint64_t cigar_cap,
              const genasm_launch* launch, void* stream, bool noalloc) {
    RoctxRange range(noalloc ? "genasm_batch_align_dev_noalloc" : "genasm_batch_align_dev");
    if (!ctx) return GENASM_E_INVAL;
    if (!valid_wko(k, W, O)) return set_err(ctx, GENASM_E_INVAL, "W must be in [2,64], O in [0,W-1], k >= 0");
    if (n_pairs == 0) return GENASM_OK;
    if (n_pairs > 0xffffffffull) return set_err(ctx, GENASM_E_INVAL, "too many pairs");
    if (!d_read_off || !d_ref_off || !d_out || (!d_reads2b && total_read_bases) ||
        (!d_refs2b && total_ref_bases) || (!d_cigar && cigar_cap))
        return set_err(ctx, GENASM_E_INVAL, "null pointer");
    if (cigar_cap < total_read_bases + total_ref_bases)
        return set_err(ctx, GENASM_E_NOSPACE, "cigar_cap below total read + reference bases");
    genasm_launch L;
    if (!launch && !ctx->tune.empty()) {
        auto it = ctx->tune.find(tune_key(n_pairs, total_read_bases, k, W, O));
        if (it != ctx->tune.end()) launch = &it->second.launch;
    }
    int rc = resolve_launch(launch, &L);
    if (rc) return set_err(ctx, rc, "bad launch parameters");
    if (noalloc && L.form == GENASM_FORM_UNIMPROVED)
        return set_err(ctx, GENASM_E_INVAL,
                       "the no-allocation call runs the plain and batched forms only");
    if (noalloc && !ctx->static_scratch)
        return set_err(ctx, GENASM_E_DEVICE, "no static scratch address on this device");
    hipStream_t s = (hipStream_t)stream;  // NULL: the null stream
    CHECK_HIP(ctx, hipSetDevice(ctx->device));
    if (!noalloc) {
        // a call recorded into a graph pins the context's buffers
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        CHECK_HIP(ctx, hipStreamIsCapturing(s, &cs));
        if (cs != hipStreamCaptureStatusNone) ctx->pinned = true;
    }
    const bool profiling = ctx->profiling && !noalloc;
    const bool counters = profiling && ctx->prof_counters;

    AlignParams p{};
    p.reads = d_reads2b;
    p.read_off = d_read_off;
    p.refs = d_refs2b;
    p.ref_off = d_ref_off;
    p.n_pairs = n_pairs;
    p.K = std::min(k, W);
    p.W = W;
    p.L = W - O;
    p.stride = p.L + 2;
    p.out = d_out;
    p.cigar = d_cigar;
    p.cigar_cap = cigar_cap;

    // Bit planes of both streams (window kernels): the context's plane buffer,
    // or the start of the static scratch.
    const uint64_t rw = plane_words(total_read_bases), fw = plane_words(total_ref_bases);
    const size_t plane_bytes = (size_t)(2 * rw + 2 * fw) * 8;
    char* plane_base;
    if (noalloc) {
        plane_base = static_cast<char*>(ctx->static_scratch);
    } else {
        rc = ensure(ctx, &ctx->planes, &ctx->planes_cap, plane_bytes);
        if (rc) return rc;
        plane_base = ctx->planes;
    }
    {
        unsigned long long* pw = reinterpret_cast<unsigned long long*>(plane_base);
        p.read_lo = pw;
        p.read_hi = pw + rw;
        p.ref_lo = pw + 2 * rw;
        p.ref_hi = pw + 2 * rw + fw;
        p.planes_from_off0 = 1;
    }
    auto too_big = [&](size_t need) {
        return set_err(ctx, GENASM_E_SCRATCH,
                       ("the batch needs " + std::to_string(need) +
                        " bytes of device scratch; the no-allocation call has " +
                        std::to_string((size_t)GENASM_NOALLOC_SCRATCH_BYTES))
                           .c_str());
    };
    if (noalloc && plane_bytes > (size_t)GENASM_NOALLOC_SCRATCH_BYTES) return too_big(plane_bytes);

    if (profiling) {
        if (counters) {
            const size_t words = (size_t)n_pairs * kStatCount;
            rc = ensure(ctx, &ctx->stats, &ctx->stats_cap, words * 8);
            if (rc) return rc;
            p.stats = reinterpret_cast<unsigned long long*>(ctx->stats);
            CHECK_HIP(ctx, launch_fill_u64(p.stats, words, 0ull, s));
        }
        ctx->prof_pairs = counters ? n_pairs : 0;
        ctx->prof_form = L.form;
        ctx->have_profile = true;
    }
    auto mark = [&](int i) -> hipError_t {
        return profiling ? hipEventRecord(ctx->ev[i], s) : hipSuccess;
    };
    auto planes = [&]() -> hipError_t {
        hipError_t e = launch_planes(d_reads2b, d_read_off, total_read_bases,
                                     const_cast<unsigned long long*>(p.read_lo),
                                     const_cast<unsigned long long*>(p.read_hi), s);
        if (e != hipSuccess) return e;
        return launch_planes(d_refs2b, d_ref_off, total_ref_bases,
                             const_cast<unsigned long long*>(p.ref_lo),
                             const_cast<unsigned long long*>(p.ref_hi), s);
    };
#if defined(GENASM_DEBUG)
    // debug builds: per-pair audit words, cleared before the kernels run (the
    // no-allocation form runs without them)
    if (!noalloc && L.form != GENASM_FORM_UNIMPROVED) {
        rc = ensure(ctx, &ctx->dbg, &ctx->dbg_cap, n_pairs * sizeof(uint32_t));
        if (rc) return rc;
        p.audit = reinterpret_cast<uint32_t*>(ctx->dbg);
        CHECK_HIP(ctx, launch_zero_u32(p.audit, n_pairs, s));
    }
#endif
    if (L.form == GENASM_FORM_UNIMPROVED) {
        p.lds_rows = 64;
        rc = ensure(ctx, &ctx->unimp, &ctx->unimp_cap, unimproved_table_words(n_pairs) * 8);
        if (rc) return rc;
        CHECK_HIP(ctx, mark(0));
        CHECK_HIP(ctx, planes());
        CHECK_HIP(ctx, mark(1));
        CHECK_HIP(ctx, mark(2));
        CHECK_HIP(ctx, launch_unimproved(p, reinterpret_cast<unsigned long long*>(ctx->unimp), s));
        CHECK_HIP(ctx, mark(3));
        return GENASM_OK;
    }
    if (L.form == GENASM_FORM_PLAIN) {
        p.lds_rows = 64;
        CHECK_HIP(ctx, mark(0));
        CHECK_HIP(ctx, planes());
        CHECK_HIP(ctx, mark(1));
        CHECK_HIP(ctx, mark(2));
        CHECK_HIP(ctx, launch_plain(p, s));
        CHECK_HIP(ctx, launch_audit(p, 0, s));  // debug builds only
        CHECK_HIP(ctx, mark(3));
        return GENASM_OK;
    }

    // Batched: scratch layout.
    p.lds_rows = L.lds_rows;
    p.hard_row = L.hard_row;
    p.hard_lanes = L.hard_lanes;
    p.tb_prefetch = L.tb_prefetch;
    p.hard_share = L.hard_share;
    p.route = 1;
    // compact groups (32-bit table slices) when both queues run 16-lane groups
    p.compact = L.table_bits == 32 && L.hard_lanes == 16 && L.group_lanes == 16;
    const int SG = L.search_lanes;
    // more resident search workgroups than 8 per CU make smaller chunks (each
    // rescanning m1 + 64 columns past its end) and measured slower
    const int search_blocks = ctx->num_cus * L.search_per_cu;
    const int spill_rows = p.compact ? kCompactSpillRows : 64 - L.lds_rows;
    // Search chunks: at least kBatchSearchChunk columns, and large enough that
    // the batch makes about two items per search group (counted at 8 search
    // workgroups per CU), so that a long reference splits only when the groups
    // would otherwise sit idle.
    {
        const uint64_t groups = (uint64_t)ctx->num_cus * 8 * (64 / SG);
        const uint64_t want = (total_ref_bases + 2 * groups - 1) / (2 * groups);
        p.search_chunk = (uint32_t)std::min<uint64_t>(
            std::max<uint64_t>(kBatchSearchChunk, (want + 1023) / 1024 * 1024), 1u << 30);
    }
    const uint64_t item_cap = search_item_cap(n_pairs, total_ref_bases, p.search_chunk);
    auto carve = [&](Carver& c, uint64_t workers) {
        p.search = c.take<SearchOut>(n_pairs);
        p.counters = c.take<uint32_t>(kCounterCount);
        p.search_key = c.take<unsigned long long>(n_pairs);
        uint64_t* items = c.take<uint64_t>(2 * item_cap);
        p.easy_list = c.take<uint32_t>(n_pairs);
        p.hard_list = c.take<uint32_t>(n_pairs);
        p.spill = spill_rows > 0 ? c.take<unsigned long long>(spill_words(workers, spill_rows)) : nullptr;
        uint32_t* hist = c.take<uint32_t>(kLptBuckets);
        uint32_t* order = c.take<uint32_t>(n_pairs);
        return std::make_tuple(items, hist, order);
    };
    // scratch bytes with `per_cu` window workgroups per CU (the static
    // scratch holds the planes first)
    const size_t base_off = noalloc ? align_up(plane_bytes, 256) : 0;
    auto scratch_need = [&](int per_cu) {
        Carver dry{nullptr};
        dry.off = base_off;
        carve(dry, (uint64_t)ctx->num_cus * per_cu * 4);
        return dry.off + 256;
    };
    int per_cu = L.workers_per_cu;
    if (per_cu == 0) {
        // as many as stay resident together (LDS and registers), so that no
        // workgroup of the persistent grid waits for another to finish; without
        // allocation, as many of those as the static scratch holds
        per_cu = std::max(1, std::min(16, windows_blocks_per_cu(p)));
        while (noalloc && per_cu > 1 && scratch_need(per_cu) > (size_t)GENASM_NOALLOC_SCRATCH_BYTES)
            --per_cu;
    }
    const int win_blocks = ctx->num_cus * per_cu;
    const uint64_t workers = (uint64_t)win_blocks * 4;
    const size_t need = scratch_need(per_cu);
    char* base;
    if (noalloc) {
        if (need > (size_t)GENASM_NOALLOC_SCRATCH_BYTES) return too_big(need);
        base = static_cast<char*>(ctx->static_scratch);
    } else {
        rc = ensure(ctx, &ctx->scratch, &ctx->scratch_cap, need);
        if (rc) return rc;
        base = ctx->scratch;
    }
    if (profiling) ctx->prof_window_blocks = win_blocks;
    Carver real{base};
    real.off = base_off;
    auto [items, hist, order] = carve(real, workers);

    CHECK_HIP(ctx, mark(0));
    CHECK_HIP(ctx, planes());
    if (L.lpt_order) {
        CHECK_HIP(ctx, launch_lpt_order(d_read_off, n_pairs, hist, order, s));
        p.order = order;
    }
    // Start search over reference chunks: the items of every pair (longest
    // reads first when ordered), stage 0 with 16 rows, stages 1-2 with 32 and 64
    // rows for the items that found no hit, then each pair's outcome and queue.
    CHECK_HIP(ctx, mark(1));
    p.list_in = p.order;
    CHECK_HIP(ctx, launch_init_counters(p.counters, (uint32_t)n_pairs, s));
    p.items_out = items;
    CHECK_HIP(ctx, launch_search_items(p, (uint32_t)n_pairs, s));
    p.list_slot = 0;
    p.items_in = items;
    p.items_out = items + item_cap;
    if (SG == 64) {
        CHECK_HIP(ctx, launch_search(p, 64, 1, search_blocks, s));
    } else {
        CHECK_HIP(ctx, launch_search(p, 16, 1, search_blocks, s));
        p.items_in = items + item_cap;
        p.items_out = items;
        p.list_slot = 1;
        CHECK_HIP(ctx, launch_search(p, 16, 2, search_blocks, s));
        p.items_in = items;
        p.items_out = items + item_cap;  // never written: 4 rows per lane cover all 64 rows
        p.list_slot = 2;
        CHECK_HIP(ctx, launch_search(p, 16, 4, search_blocks, s));
    }
    CHECK_HIP(ctx, launch_search_finalize(p, (uint32_t)n_pairs, s));
    // Windows: persistent workers pull pairs (longest first) from the queue.
    CHECK_HIP(ctx, mark(2));
    p.list_in = nullptr;
    p.items_in = nullptr;
    p.items_out = nullptr;
    CHECK_HIP(ctx, launch_windows(p, win_blocks, s));
    CHECK_HIP(ctx, launch_audit(p, 1, s));  // debug builds only
    CHECK_HIP(ctx, mark(3));
    return GENASM_OK;
}

}  // namespace

extern "C" {

int genasm_batch_align_dev(genasm_ctx* ctx, const uint8_t* d_reads2b, const uint64_t* d_read_off,
                           const uint8_t* d_refs2b, const uint64_t* d_ref_off, uint64_t n_pairs,
                           uint64_t total_read_bases, uint64_t total_ref_bases,
                           int32_t k, int32_t W, int32_t O,
                           genasm_result* d_out, uint32_t* d_cigar, uint64_t cigar_cap,
                           const genasm_launch* launch, void* stream) {
    return align_dev(ctx, d_reads2b, d_read_off, d_refs2b, d_ref_off, n_pairs, total_read_bases,
                     total_ref_bases, k, W, O, d_out, d_cigar, cigar_cap, launch, stream, false);
}

int genasm_batch_align_dev_noalloc(genasm_ctx* ctx, const uint8_t* d_reads2b,
                                   const uint64_t* d_read_off, const uint8_t* d_refs2b,
                                   const uint64_t* d_ref_off, uint64_t n_pairs,
                                   uint64_t total_read_bases, uint64_t total_ref_bases,
                                   int32_t k, int32_t W, int32_t O,
                                   genasm_result* d_out, uint32_t* d_cigar, uint64_t cigar_cap,
                                   const genasm_launch* launch, void* stream) {
    return align_dev(ctx, d_reads2b, d_read_off, d_refs2b, d_ref_off, n_pairs, total_read_bases,
                     total_ref_bases, k, W, O, d_out, d_cigar, cigar_cap, launch, stream, true);
}

int genasm_autotune_dev(genasm_ctx* ctx, const uint8_t* d_reads2b, const uint64_t* d_read_off,
                        const uint8_t* d_refs2b, const uint64_t* d_ref_off, uint64_t n_pairs,
                        uint64_t total_read_bases, uint64_t total_ref_bases,
                        int32_t k, int32_t W, int32_t O, genasm_result* d_out, uint32_t* d_cigar,
                        uint64_t cigar_cap, int32_t reps, void* stream, genasm_launch* best,
                        float* best_ms) {
    if (!ctx || !best) return GENASM_E_INVAL;
    if (reps < 1) reps = 1;
    hipStream_t s = (hipStream_t)stream;
    CHECK_HIP(ctx, hipSetDevice(ctx->device));
    // Candidates: lanes per pair for the decoy-like queue (16: four pairs per
    // wavefront; 64: one) and its start-row threshold, table rows kept in LDS
    // per 16-lane group (the rest spill), and resident workers per CU.
    std::vector<genasm_launch> cands;
    auto add = [&](int hard_row, int hard_lanes, int lds_rows, int workers, int search_lanes,
                   int table_bits) {
        genasm_launch c;
        genasm_default_launch(GENASM_FORM_BATCHED, &c);
        c.hard_row = hard_row;
        c.hard_lanes = hard_lanes;
        c.lds_rows = lds_rows;
        c.workers_per_cu = workers;
        c.search_lanes = search_lanes;
        c.table_bits = table_bits;
        cands.push_back(c);
    };
    // compact groups: the hard-queue threshold, resident workers, search lanes
    for (int hr : {12, 16, 24, 65}) add(hr, 16, 16, 0, 16, 32);
    add(16, 16, 16, 8, 16, 32);
    add(16, 16, 16, 0, 64, 32);
    for (int spc : {4, 16}) {
        genasm_launch c;
        genasm_default_launch(GENASM_FORM_BATCHED, &c);
        c.search_per_cu = spc;
        cands.push_back(c);
    }
    // 64-bit tables: LDS rows, lanes per hard pair and their threshold
    add(16, 16, 16, 0, 16, 64);
    add(16, 16, 32, 0, 16, 64);
    add(16, 64, 16, 0, 16, 64);
    for (int hr : {12, 16, 24}) add(hr, 32, 16, 0, 16, 64);
    add(-1, 64, 16, 0, 16, 64);  // every pair one per wavefront
    {
        genasm_launch c;
        genasm_default_launch(GENASM_FORM_BATCHED, &c);
        c.tb_prefetch = 1;
        cands.push_back(c);
        genasm_default_launch(GENASM_FORM_BATCHED, &c);
        for (int share : {25, 75, 100}) {
            c.hard_share = share;
            cands.push_back(c);
        }
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    CHECK_HIP(ctx, hipEventCreate(&e0));
    CHECK_HIP(ctx, hipEventCreate(&e1));
    int rc = GENASM_OK;
    float best_t = 1e30f;
    for (const genasm_launch& c : cands) {
        // a first run sizes the scratch for this shape, then timed runs
        rc = genasm_batch_align_dev(ctx, d_reads2b, d_read_off, d_refs2b, d_ref_off, n_pairs,
                                    total_read_bases, total_ref_bases, k, W, O, d_out,
                                    d_cigar, cigar_cap, &c, stream);
        if (rc) break;
        float t_min = 1e30f;
        for (int r = 0; r < reps && !rc; ++r) {
            if (hipEventRecord(e0, s) != hipSuccess) { rc = GENASM_E_DEVICE; break; }
            rc = genasm_batch_align_dev(ctx, d_reads2b, d_read_off, d_refs2b, d_ref_off, n_pairs,
                                        total_read_bases, total_ref_bases, k, W, O,
                                        d_out, d_cigar, cigar_cap, &c, stream);
            float ms = 0.f;
            if (!rc && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                        hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
                rc = GENASM_E_DEVICE;
            t_min = std::min(t_min, ms);
        }
        if (rc) break;
        if (t_min < best_t) {
            best_t = t_min;
            *best = c;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc == GENASM_E_DEVICE ? set_err(ctx, rc, "autotune timing failed") : rc;
    ctx->tune[tune_key(n_pairs, total_read_bases, k, W, O)] = genasm_ctx::Tuned{*best, best_t};
    if (best_ms) *best_ms = best_t;
    return GENASM_OK;
}

int genasm_tune_cache_save(genasm_ctx* ctx, const char* path) {
    if (!ctx || !path) return GENASM_E_INVAL;
    FILE* f = std::fopen(path, "w");
    if (!f) return set_err(ctx, GENASM_E_INVAL, "cannot open tune cache file for writing");
    std::fprintf(f, "# key form group_lanes search_lanes lds_rows workers_per_cu lpt_order hard_row "
                    "hard_lanes tb_prefetch hard_share table_bits search_per_cu ms\n");
    for (const auto& kv : ctx->tune) {
        const genasm_launch& L = kv.second.launch;
        std::fprintf(f, "%s %d %d %d %d %d %d %d %d %d %d %d %d %.4f\n", kv.first.c_str(), L.form,
                     L.group_lanes, L.search_lanes, L.lds_rows, L.workers_per_cu, L.lpt_order,
                     L.hard_row, L.hard_lanes, L.tb_prefetch, L.hard_share, L.table_bits,
                     L.search_per_cu, kv.second.ms);
    }
    const bool ok = std::fclose(f) == 0;
    return ok ? GENASM_OK : set_err(ctx, GENASM_E_INVAL, "writing the tune cache failed");
}

int genasm_tune_cache_load(genasm_ctx* ctx, const char* path) {
    if (!ctx || !path) return GENASM_E_INVAL;
    FILE* f = std::fopen(path, "r");
    if (!f) return set_err(ctx, GENASM_E_INVAL, "cannot open tune cache file");
    char line[512];
    int rc = GENASM_OK;
    while (std::fgets(line, sizeof line, f)) {
        if (line[0] == '#' || line[0] == '\n') continue;
        char key[256];
        genasm_launch L{};
        float ms = 0.f;
        const int got = std::sscanf(line, "%255s %d %d %d %d %d %d %d %d %d %d %d %d %f", key,
                                    &L.form, &L.group_lanes, &L.search_lanes, &L.lds_rows,
                                    &L.workers_per_cu, &L.lpt_order, &L.hard_row, &L.hard_lanes,
                                    &L.tb_prefetch, &L.hard_share, &L.table_bits,
                                    &L.search_per_cu, &ms);
        genasm_launch chk;
        if (got != 14 || resolve_launch(&L, &chk) != GENASM_OK) { rc = GENASM_E_INVAL; break; }
        ctx->tune[key] = genasm_ctx::Tuned{L, ms};
    }
    std::fclose(f);
    return rc ? set_err(ctx, rc, "malformed tune cache line") : GENASM_OK;
}

int genasm_tune_cache_size(genasm_ctx* ctx) { return ctx ? (int)ctx->tune.size() : GENASM_E_INVAL; }

int genasm_profile_enable(genasm_ctx* ctx, int on) {
    if (!ctx) return GENASM_E_INVAL;
    CHECK_HIP(ctx, hipSetDevice(ctx->device));
    if (on) {
        for (hipEvent_t& e : ctx->ev)
            if (!e) CHECK_HIP(ctx, hipEventCreate(&e));
    }
    if (on < 0 || on > 2) return set_err(ctx, GENASM_E_INVAL, "profiling level must be 0, 1 or 2");
    ctx->profiling = on != 0;
    ctx->prof_counters = on == 1;
    return GENASM_OK;
}

int genasm_profile_pairs(genasm_ctx* ctx, uint64_t* out, uint64_t max_words, uint64_t* words) {
    if (!ctx || !words) return GENASM_E_INVAL;
    if (!ctx->have_profile) return set_err(ctx, GENASM_E_INVAL, "no profiled call yet");
    const uint64_t n = ctx->prof_pairs * kStatCount;
    *words = n;
    if (!out || max_words < n) return n ? GENASM_E_NOSPACE : GENASM_OK;
    CHECK_HIP(ctx, hipSetDevice(ctx->device));
    CHECK_HIP(ctx, hipEventSynchronize(ctx->ev[3]));
    if (n) CHECK_HIP(ctx, hipMemcpy(out, ctx->stats, n * 8, hipMemcpyDeviceToHost));
    return GENASM_OK;
}

int genasm_profile_read(genasm_ctx* ctx, genasm_profile* out) {
    if (!ctx || !out) return GENASM_E_INVAL;
    if (!ctx->have_profile) return set_err(ctx, GENASM_E_INVAL, "no profiled call yet");
    CHECK_HIP(ctx, hipSetDevice(ctx->device));
    CHECK_HIP(ctx, hipEventSynchronize(ctx->ev[3]));
    std::memset(out, 0, sizeof(*out));
    CHECK_HIP(ctx, hipEventElapsedTime(&out->total_ms, ctx->ev[0], ctx->ev[3]));
    CHECK_HIP(ctx, hipEventElapsedTime(&out->order_ms, ctx->ev[0], ctx->ev[1]));
    CHECK_HIP(ctx, hipEventElapsedTime(&out->search_ms, ctx->ev[1], ctx->ev[2]));
    CHECK_HIP(ctx, hipEventElapsedTime(&out->windows_ms, ctx->ev[2], ctx->ev[3]));
    const size_t words = (size_t)ctx->prof_pairs * kStatCount;
    std::vector<unsigned long long> st(words);
    if (words)
        CHECK_HIP(ctx, hipMemcpy(st.data(), ctx->stats, words * 8, hipMemcpyDeviceToHost));
    uint64_t sum[kStatCount] = {0};
    for (size_t i = 0; i < words; ++i) sum[i % kStatCount] += st[i];
    out->n_pairs = ctx->prof_pairs;
    out->window_word_ops = sum[kStatWindowWordOps];
    out->search_word_ops = sum[kStatSearchWordOps];
    out->window_cells = sum[kStatWindowCells];
    out->search_cells = sum[kStatSearchCells];
    out->table_words = sum[kStatTableWords];
    out->tb_reads = sum[kStatTbReads];
    out->window_lane_steps = sum[kStatWindowLaneSteps];
    out->search_lane_steps = sum[kStatSearchLaneSteps];
    out->windows = sum[kStatWindows];
    out->dc_cycles = sum[kStatDcCycles];
    out->tb_cycles = sum[kStatTbCycles];
    out->pair_cycles = sum[kStatPairCycles];
    out->window_workgroups = (uint64_t)ctx->prof_window_blocks;
    return GENASM_OK;
}

int genasm_filter_dev(genasm_ctx* ctx, const uint8_t* d_reads2b, const uint64_t* d_read_off,
                      const uint8_t* d_refs2b, const uint64_t* d_ref_off, uint64_t n_pairs,
                      uint32_t max_read_len, int32_t k, int32_t* d_dist, uint32_t* d_start,
                      void* stream) {
    if (!ctx) return GENASM_E_INVAL;
    if (k < 0 || k > 63) return set_err(ctx, GENASM_E_INVAL, "filter k must be in [0, 63]");
    if (n_pairs == 0) return GENASM_OK;
    if (n_pairs > 0xffffffffull) return set_err(ctx, GENASM_E_INVAL, "too many pairs");
    if (!d_read_off || !d_ref_off || !d_dist || !d_start)
        return set_err(ctx, GENASM_E_INVAL, "null pointer");
    if (filter_words(max_read_len) == 0)
        return set_err(ctx, GENASM_E_TOOLONG, "filter reads are limited to 1024 bases");
    CHECK_HIP(ctx, hipSetDevice(ctx->device));
    CHECK_HIP(ctx, launch_filter(d_reads2b, d_read_off, d_refs2b, d_ref_off, n_pairs, max_read_len,
                                 k, d_dist, d_start, (hipStream_t)stream));
    return GENASM_OK;
}

int genasm_filter(genasm_ctx* ctx, const char* reads, const uint64_t* read_off, const char* refs,
                  const uint64_t* ref_off, uint64_t n_pairs, int32_t k, int32_t* dist,
                  uint32_t* start) {
    if (!ctx) return GENASM_E_INVAL;
    if (k < 0 || k > 63) return set_err(ctx, GENASM_E_INVAL, "filter k must be in [0, 63]");
    if (!read_off || !ref_off || ((!dist || !start) && n_pairs))
        return set_err(ctx, GENASM_E_INVAL, "null pointer");
    int rc = check_offsets(read_off, n_pairs, UINT64_MAX);
    if (!rc) rc = check_offsets(ref_off, n_pairs, UINT64_MAX);
    if (rc) return set_err(ctx, rc, "bad offsets");
    if (n_pairs == 0) return GENASM_OK;
    if ((!reads && read_off[n_pairs] > read_off[0]) || (!refs && ref_off[n_pairs] > ref_off[0]))
        return set_err(ctx, GENASM_E_INVAL, "null sequence pointer");
    const uint64_t nr = read_off[n_pairs] - read_off[0];
    const uint64_t nf = ref_off[n_pairs] - ref_off[0];
    std::vector<uint64_t> roff(n_pairs + 1), foff(n_pairs + 1);
    uint32_t max_read = 0;
    for (uint64_t i = 0; i <= n_pairs; ++i) {
        roff[i] = read_off[i] - read_off[0];
        foff[i] = ref_off[i] - ref_off[0];
        if (i) max_read = std::max<uint32_t>(max_read, (uint32_t)std::min<uint64_t>(roff[i] - roff[i - 1], 0xffffffffull));
    }
    if (filter_words(max_read) == 0)
        return set_err(ctx, GENASM_E_TOOLONG, "filter reads are limited to 1024 bases");
    CHECK_HIP(ctx, hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;
    auto carve = [&](Carver& c) {
        struct B {
            char *ar, *af;
            uint8_t *pr, *pf;
            uint64_t *or_, *of;
            int32_t* dist;
            uint32_t *start, *bad;
        } b;
        b.ar = c.take<char>(nr + 1);
        b.af = c.take<char>(nf + 1);
        b.pr = c.take<uint8_t>(nr / 4 + 2);
        b.pf = c.take<uint8_t>(nf / 4 + 2);
        b.or_ = c.take<uint64_t>(n_pairs + 1);
        b.of = c.take<uint64_t>(n_pairs + 1);
        b.dist = c.take<int32_t>(n_pairs);
        b.start = c.take<uint32_t>(n_pairs);
        b.bad = c.take<uint32_t>(2);
        return b;
    };
    Carver dry{nullptr};
    carve(dry);
    rc = ensure(ctx, &ctx->stage, &ctx->stage_cap, dry.off + 256);
    if (rc) return rc;
    Carver real{ctx->stage};
    auto b = carve(real);
    CHECK_HIP(ctx, hipMemsetAsync(b.bad, 0, 2 * sizeof(uint32_t), s));
    if (nr) CHECK_HIP(ctx, hipMemcpyAsync(b.ar, reads + read_off[0], nr, hipMemcpyHostToDevice, s));
    if (nf) CHECK_HIP(ctx, hipMemcpyAsync(b.af, refs + ref_off[0], nf, hipMemcpyHostToDevice, s));
    CHECK_HIP(ctx, hipMemcpyAsync(b.or_, roff.data(), (n_pairs + 1) * 8, hipMemcpyHostToDevice, s));
    CHECK_HIP(ctx, hipMemcpyAsync(b.of, foff.data(), (n_pairs + 1) * 8, hipMemcpyHostToDevice, s));
    CHECK_HIP(ctx, launch_pack(b.ar, nr, b.pr, b.bad, s));
    CHECK_HIP(ctx, launch_pack(b.af, nf, b.pf, b.bad, s));
    uint32_t bad = 0;
    CHECK_HIP(ctx, hipMemcpyAsync(&bad, b.bad, sizeof(bad), hipMemcpyDeviceToHost, s));
    CHECK_HIP(ctx, hipStreamSynchronize(s));
    if (bad) return set_err(ctx, GENASM_E_ALPHABET, "sequence byte outside ACGTacgt");
    CHECK_HIP(ctx, launch_filter(b.pr, b.or_, b.pf, b.of, n_pairs, max_read, k, b.dist, b.start, s));
    CHECK_HIP(ctx, hipMemcpyAsync(dist, b.dist, n_pairs * 4, hipMemcpyDeviceToHost, s));
    CHECK_HIP(ctx, hipMemcpyAsync(start, b.start, n_pairs * 4, hipMemcpyDeviceToHost, s));
    CHECK_HIP(ctx, hipStreamSynchronize(s));
    return GENASM_OK;
}

int genasm_batch_align(genasm_ctx* ctx, const char* reads, const uint64_t* read_off,
                       const char* refs, const uint64_t* ref_off, uint64_t n_pairs,
                       int32_t k, int32_t W, int32_t O, genasm_result* out, char* cigar_buf,
                       uint64_t cigar_cap, uint64_t* cigar_needed, const genasm_launch* launch) {
    RoctxRange range("genasm_batch_align");
    if (!ctx) return GENASM_E_INVAL;
    if (!valid_wko(k, W, O)) return set_err(ctx, GENASM_E_INVAL, "W must be in [2,64], O in [0,W-1], k >= 0");
    if (!read_off || !ref_off || (!out && n_pairs) || !cigar_needed || (!cigar_buf && cigar_cap))
        return set_err(ctx, GENASM_E_INVAL, "null pointer");
    int rc = check_offsets(read_off, n_pairs, UINT64_MAX);
    if (!rc) rc = check_offsets(ref_off, n_pairs, UINT64_MAX);
    if (rc) return set_err(ctx, rc, "bad offsets");
    *cigar_needed = 0;
    if (n_pairs == 0) return GENASM_OK;
    if ((!reads && read_off[n_pairs] > read_off[0]) || (!refs && ref_off[n_pairs] > ref_off[0]))
        return set_err(ctx, GENASM_E_INVAL, "null sequence pointer");
    genasm_launch L;
    rc = resolve_launch(launch, &L);
    if (rc) return set_err(ctx, rc, "bad launch parameters");
    CHECK_HIP(ctx, hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;

    const uint64_t nr = read_off[n_pairs] - read_off[0];
    const uint64_t nf = ref_off[n_pairs] - ref_off[0];
    std::vector<uint64_t> roff(n_pairs + 1), foff(n_pairs + 1);
    for (uint64_t i = 0; i <= n_pairs; ++i) {
        roff[i] = read_off[i] - read_off[0];
        foff[i] = ref_off[i] - ref_off[0];
    }
    Carver dry{nullptr};
    auto carve = [&](Carver& c) {
        struct B {
            char *ar, *af;
            uint8_t *pr, *pf;
            uint64_t *or_, *of, *dst_off;
            genasm_result* res;
            uint32_t *cig, *cig2, *bad;
        } b;
        b.ar = c.take<char>(nr + 1);
        b.af = c.take<char>(nf + 1);
        b.pr = c.take<uint8_t>(nr / 4 + 2);
        b.pf = c.take<uint8_t>(nf / 4 + 2);
        b.or_ = c.take<uint64_t>(n_pairs + 1);
        b.of = c.take<uint64_t>(n_pairs + 1);
        b.dst_off = c.take<uint64_t>(n_pairs + 1);
        b.res = c.take<genasm_result>(n_pairs);
        b.cig = c.take<uint32_t>(nr + nf + 1);
        b.cig2 = c.take<uint32_t>(nr + nf + 1);
        b.bad = c.take<uint32_t>(2);
        return b;
    };
    carve(dry);
    rc = ensure(ctx, &ctx->stage, &ctx->stage_cap, dry.off + 256);
    if (rc) return rc;
    Carver real{ctx->stage};
    auto b = carve(real);

    CHECK_HIP(ctx, hipMemsetAsync(b.bad, 0, 2 * sizeof(uint32_t), s));
    if (nr) CHECK_HIP(ctx, hipMemcpyAsync(b.ar, reads + read_off[0], nr, hipMemcpyHostToDevice, s));
    if (nf) CHECK_HIP(ctx, hipMemcpyAsync(b.af, refs + ref_off[0], nf, hipMemcpyHostToDevice, s));
    CHECK_HIP(ctx, hipMemcpyAsync(b.or_, roff.data(), (n_pairs + 1) * 8, hipMemcpyHostToDevice, s));
    CHECK_HIP(ctx, hipMemcpyAsync(b.of, foff.data(), (n_pairs + 1) * 8, hipMemcpyHostToDevice, s));
    CHECK_HIP(ctx, launch_pack(b.ar, nr, b.pr, b.bad, s));
    CHECK_HIP(ctx, launch_pack(b.af, nf, b.pf, b.bad, s));
    uint32_t bad = 0;
    CHECK_HIP(ctx, hipMemcpyAsync(&bad, b.bad, sizeof(bad), hipMemcpyDeviceToHost, s));
    CHECK_HIP(ctx, hipStreamSynchronize(s));
    if (bad) return set_err(ctx, GENASM_E_ALPHABET, "sequence byte outside ACGTacgt");

    rc = genasm_batch_align_dev(ctx, b.pr, b.or_, b.pf, b.of, n_pairs, nr, nf, k, W, O,
                                b.res, b.cig, nr + nf + 1, &L, s);
    if (rc) return rc;
    // results are staged on the host: out[] is written only when the CIGAR
    // text fits, so GENASM_E_NOSPACE leaves no partial results
    std::vector<genasm_result> res(n_pairs);
    CHECK_HIP(ctx, hipMemcpyAsync(res.data(), b.res, n_pairs * sizeof(genasm_result),
                                  hipMemcpyDeviceToHost, s));
    CHECK_HIP(ctx, hipStreamSynchronize(s));
    // Gather the CIGAR elements of all pairs into one dense buffer.
    std::vector<uint64_t> dst(n_pairs + 1, 0);
    for (uint64_t i = 0; i < n_pairs; ++i) dst[i + 1] = dst[i] + res[i].cigar_len;
    const uint64_t n_elems = dst[n_pairs];
    std::vector<uint32_t> elems(n_elems);
    if (n_elems) {
        CHECK_HIP(ctx, hipMemcpyAsync(b.dst_off, dst.data(), (n_pairs + 1) * 8,
                                      hipMemcpyHostToDevice, s));
        CHECK_HIP(ctx, launch_compact_cigar(b.res, b.dst_off, n_pairs, b.cig, b.cig2, s));
        CHECK_HIP(ctx, hipMemcpyAsync(elems.data(), b.cig2, n_elems * 4, hipMemcpyDeviceToHost, s));
        CHECK_HIP(ctx, hipStreamSynchronize(s));
    }
    // Format the text CIGARs: per-pair text lengths, their prefix sum, then
    // the text itself, each pass split over host threads by pair ranges.
    std::vector<uint64_t> tpos(n_pairs + 1, 0);
    const unsigned n_thr = (unsigned)std::max<uint64_t>(
        1, std::min<uint64_t>({(uint64_t)std::max(1u, std::thread::hardware_concurrency()), 16,
                               n_elems / 65536 + 1}));
    auto parallel = [&](auto&& body) {
        std::vector<std::thread> th;
        for (unsigned t = 1; t < n_thr; ++t)
            th.emplace_back(body, n_pairs * t / n_thr, n_pairs * (t + 1) / n_thr);
        body((uint64_t)0, n_pairs / n_thr);
        for (auto& x : th) x.join();
    };
    parallel([&](uint64_t lo, uint64_t hi) {
        for (uint64_t i = lo; i < hi; ++i) {
            uint64_t chars = 0;
            for (uint64_t e = dst[i]; e < dst[i + 1]; ++e) chars += cigar_run_chars(elems[e]);
            tpos[i + 1] = chars;
        }
    });
    for (uint64_t i = 0; i < n_pairs; ++i) tpos[i + 1] += tpos[i];
    const uint64_t need = tpos[n_pairs];
    *cigar_needed = need;
    if (need > cigar_cap) return set_err(ctx, GENASM_E_NOSPACE, "cigar_cap below the CIGAR text size");
    parallel([&](uint64_t lo, uint64_t hi) {
        for (uint64_t i = lo; i < hi; ++i) {
            char* w = cigar_buf + tpos[i];
            for (uint64_t e = dst[i]; e < dst[i + 1]; ++e) w = cigar_run_text(elems[e], w);
        }
    });
    for (uint64_t i = 0; i < n_pairs; ++i) {
        res[i].cigar_off = tpos[i];
        res[i].cigar_len = (uint32_t)(tpos[i + 1] - tpos[i]);
    }
    std::memcpy(out, res.data(), n_pairs * sizeof(genasm_result));
    return GENASM_OK;
}

}  // extern "C"
