// Serving form of the GenASM library: continuous batching of single-pair
// requests with device-resident sequences and per-pair window state.
//
// An engine thread runs device iterations on one stream. An iteration admits
// waiting requests into free slots (bounded by the slot count, the base pool
// and the CIGAR pool), uploads their packed bases (one copy, two scatter
// kernels), then runs one captured graph:
//
//   begin (counters; slot tables and fresh state of the admitted pairs)
//   -> start search of the admitted pairs -> window kernel -> finish
//
// The window kernel takes the resident pairs from two device lists: the pairs
// admitted now and those whose previous turn was cut after one window first,
// then the others. Every pair advances at least one window, and more until it
// ends or the iteration's window time has passed; the kernel itself puts each
// pair on the
// next iteration's lists or on the finished list, so the host never copies or
// scans per-slot state. The finish kernels write the finished pairs' slots and
// results into host-mapped memory and gather their CIGAR elements into one
// device buffer, which the host copies on a second stream.
//
// Two iterations can be in flight: while the device runs iteration t, the
// engine collects the output of t-1 and, when requests wait or the device is
// saturated, queues t+1 behind t. Buffers that the host writes or reads while
// an iteration runs exist twice, once per iteration parity, and so do the two
// captured graphs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <set>
#include <string>
#include <thread>
#include <vector>

#include "internal.h"
#include "range_alloc.h"
#include "trace.h"

using namespace genasm;

namespace {

uint64_t steady_ns() {
    return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

constexpr uint64_t kBaseUnit = 64;  // pool allocations in bases: whole bit-plane words
constexpr uint64_t kArenaChunk = 4ull << 20;  // pinned chunk that submissions are packed into

uint64_t round_up(uint64_t x, uint64_t a) { return (x + a - 1) / a * a; }

// Pinned host blocks, reused: a block goes back to the free list of its size
// class (powers of two from 1 MiB) when its last reference drops, in whatever
// thread that happens; up to kKeepBytes stay cached, beyond that they are
// freed. Copies between these blocks and the device run at full PCIe rate with
// no staging copy on either side.
class HostPool : public std::enable_shared_from_this<HostPool> {
  public:
    static constexpr int kMinClass = 20;
    static constexpr uint64_t kKeepBytes = 1ull << 30;
    ~HostPool() {
        for (auto& f : free_)
            for (void* p : f) (void)hipHostFree(p);
    }
    // Puts `count` blocks of `bytes` bytes (a power of two from 1 MiB) into the
    // free lists ahead of use, with their pages touched: the first write to a
    // freshly pinned page is many times slower than later ones.
    void warm(uint64_t bytes, int count) {
        std::vector<std::shared_ptr<uint8_t>> held;
        for (int i = 0; i < count; ++i) {
            std::shared_ptr<uint8_t> b = get(bytes);
            if (!b) break;
            std::memset(b.get(), 0, bytes);
            held.push_back(std::move(b));
        }
    }
    // A block of at least `bytes` bytes, or null when none can be allocated.
    std::shared_ptr<uint8_t> get(uint64_t bytes) {
        int k = kMinClass;
        while ((1ull << k) < bytes) ++k;
        if (k >= 48) return nullptr;
        void* p = nullptr;
        {
            std::lock_guard<std::mutex> lk(mu_);
            if (!free_[k].empty()) {
                p = free_[k].back();
                free_[k].pop_back();
                cached_ -= 1ull << k;
            }
        }
        if (!p && hipHostMalloc(&p, 1ull << k, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        std::shared_ptr<HostPool> self = shared_from_this();
        return std::shared_ptr<uint8_t>(static_cast<uint8_t*>(p),
                                        [self, k](uint8_t* q) { self->put(q, k); });
    }

  private:
    void put(void* p, int k) {
        {
            std::lock_guard<std::mutex> lk(mu_);
            if (cached_ + (1ull << k) <= kKeepBytes) {
                free_[k].push_back(p);
                cached_ += 1ull << k;
                return;
            }
        }
        (void)hipHostFree(p);
    }
    std::mutex mu_;
    std::vector<void*> free_[48];
    uint64_t cached_ = 0;
};

// A queued request: its read's packed bytes, then its reference's, at `off`
// in a pinned block that it shares with the requests submitted around it.
struct Request {
    std::shared_ptr<uint8_t> block;
    uint64_t off = 0;
    uint32_t m = 0, n = 0;
    uint64_t tag = 0, submit_ns = 0;
    uint64_t read_bytes() const { return ((uint64_t)m + 3) / 4; }
    uint64_t bytes() const { return read_bytes() + ((uint64_t)n + 3) / 4; }
    const uint8_t* data() const { return block.get() + off; }
};

// A finished request on its way to the caller: the CIGAR elements stay in the
// iteration's pinned completion block until a poll copies or formats them (in
// the polling thread, not the engine's).
struct DoneRec {
    uint64_t tag;
    genasm_result result;  // cigar_off: element offset in `block`; cigar_len: elements
    uint64_t submit_ns, admit_ns, done_ns;
    std::shared_ptr<uint8_t> block;
    const uint32_t* elements() const {
        return reinterpret_cast<const uint32_t*>(block.get()) + result.cigar_off;
    }
};

struct Slot {
    uint64_t tag = 0, submit_ns = 0, admit_ns = 0;
    uint64_t bstart = 0, blen = 0;  // base pool range (bases): the read, then the reference
    uint32_t bh = 0, ch = 0;        // their allocator handles
    uint64_t fstart = 0;            // where the reference starts in it
    uint64_t cstart = 0, clen = 0;  // CIGAR pool range (elements)
};

template <class T>
T* host_alloc(size_t n, unsigned flags = hipHostMallocDefault) {
    void* p = nullptr;
    if (hipHostMalloc(&p, std::max<size_t>(n, 1) * sizeof(T), flags) != hipSuccess) return nullptr;
    return static_cast<T*>(p);
}

template <class T>
T* dev_alloc(size_t n) {
    // failure injection for tests of the error path (see runtime.hip)
    const char* fail = std::getenv("GENASM_FAIL_ALLOC");
    if (fail && fail[0] == '1') return nullptr;
    void* p = nullptr;
    if (hipMalloc(&p, std::max<size_t>(n, 1) * sizeof(T)) != hipSuccess) return nullptr;
    return static_cast<T*>(p);
}

// Buffers of one iteration parity.
struct IterBufs {
    // upload staging (pinned host) and its device copy
    uint8_t *h_upload = nullptr, *d_upload = nullptr;
    uint64_t *h_up_src = nullptr, *h_up_dst = nullptr, *h_up_word = nullptr;
    uint64_t *d_up_src = nullptr, *d_up_dst = nullptr, *d_up_word = nullptr;
    uint32_t *h_up_len = nullptr, *h_up_bases = nullptr, *d_up_len = nullptr, *d_up_bases = nullptr;
    ServeAdmit *h_admit = nullptr, *d_admit = nullptr;
    uint32_t *h_params = nullptr, *d_params = nullptr;
    // window lists read by this parity's iterations (hot: advanced no window
    // last time, or admitted now; cold: the rest) and its counters block
    uint32_t *d_hot = nullptr, *d_cold = nullptr, *d_cnt = nullptr;
    // finished-pair summary, written by the device into host-mapped memory
    unsigned long long* h_hdr = nullptr;
    uint32_t* h_slot = nullptr;
    genasm_result* h_res = nullptr;
    unsigned long long* dh_hdr = nullptr;
    uint32_t* dh_slot = nullptr;
    genasm_result* dh_res = nullptr;
    // gathered CIGAR elements of the finished pairs
    uint32_t* d_gather = nullptr;
    // submission blocks the iteration's uploads read from (kept until it ends)
    std::vector<std::shared_ptr<uint8_t>> holds;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t ev_start = nullptr, ev_done = nullptr;
    hipEvent_t ev_up = nullptr;  // the iteration's uploads are done
    uint32_t n_new = 0;
};

}  // namespace

struct genasm_server {
    genasm_ctx* ctx = nullptr;
    genasm_server_config cfg{};
    AlignParams base{};   // fields common to every iteration's kernels
    int search_blocks = 0, win_blocks = 0;
    uint32_t groups = 0;  // 16-lane window groups of the persistent grid
    // s: the iterations; s_up: their uploads, which overlap the iteration
    // before; s_copy: completions to the host and the arrival count
    hipStream_t s = nullptr, s_up = nullptr, s_copy = nullptr;
    uint64_t gather_cap = 0;  // elements per gather buffer

    // device state shared by both parities
    uint8_t* d_pool = nullptr;                 // 2-bit packed bases (start search)
    unsigned long long *d_plo = nullptr, *d_phi = nullptr;  // the same bases as bit planes (windows)
    uint32_t* d_cigar = nullptr;
    uint64_t *d_read_off = nullptr, *d_ref_off = nullptr, *d_run_base = nullptr;
    uint32_t *d_read_len = nullptr, *d_ref_len = nullptr;
    genasm_result* d_out = nullptr;
    PairState* d_state = nullptr;
    SearchOut* d_search = nullptr;
    uint32_t* d_new = nullptr;               // slots admitted in the running iteration
    uint32_t *d_fin = nullptr, *d_fin_len = nullptr;
    uint64_t* d_fin_off = nullptr;
    uint64_t* d_items = nullptr;             // two start-search item lists
    unsigned long long* d_key = nullptr;     // per-slot search key
    TurnLimits* d_turn = nullptr;            // the running iteration's turn limits
    unsigned long long* d_arrivals = nullptr;  // arrival count, copied from h_arrivals
    unsigned long long* h_arrivals = nullptr;  // pinned
    uint64_t item_cap = 0;
    unsigned long long* d_spill = nullptr;
    uint64_t upload_cap = 0;
    IterBufs it[2];

    // pinned host blocks: submissions (an arena of chunks, or a block of their
    // own when large) and per-iteration completion blocks
    std::shared_ptr<HostPool> hpool = std::make_shared<HostPool>();
    std::mutex arena_mu;
    std::shared_ptr<uint8_t> arena;
    uint64_t arena_used = 0, arena_size = 0;

    // engine-thread state
    std::vector<Slot> slots;
    std::vector<uint32_t> free_slots;
    uint32_t resident = 0;
    RangeAlloc pool, cigpool;

    // shared state (mu)
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request> pending;
    uint64_t arrivals = 0;               // requests accepted so far
    bool signalled = false;              // arrivals copied to the device since the last admission
    std::deque<DoneRec> done;
    std::vector<uint64_t> slot_tag;      // resident request per slot (mu): tag,
    std::vector<uint8_t> slot_state;     // and 0 free, 1 resident, 2 resident and cancelled
    std::thread engine;
    bool stop = false;
    int error = GENASM_OK;
    std::string err_msg;
    genasm_server_stats st{};
};

namespace {

int srv_fail(genasm_server* srv, const char* what, hipError_t e) {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->error = GENASM_E_DEVICE;
    srv->err_msg = std::string(what) + ": " + hipGetErrorString(e);
    srv->cv_done.notify_all();
    return GENASM_E_DEVICE;
}

#define SRV_HIP(srv, expr)                                          \
    do {                                                            \
        hipError_t e_ = (expr);                                     \
        if (e_ != hipSuccess) return srv_fail(srv, #expr, e_);      \
    } while (0)

// The device work of one iteration of parity q (graph capture or direct launch).
hipError_t enqueue_iteration(genasm_server* srv, int q) {
    hipError_t e;
    IterBufs& b = srv->it[q];
    IterBufs& nb = srv->it[1 - q];
    const uint32_t NS = srv->cfg.max_slots;
    hipStream_t s = srv->s;
    ServeSlots slots{srv->d_read_off, srv->d_ref_off, srv->d_run_base,
                     srv->d_read_len, srv->d_ref_len, srv->d_state};
    if ((e = launch_serve_begin(b.d_cnt, nb.d_cnt, srv->d_fin_len, b.d_params, b.d_admit, slots,
                                srv->d_new, s)))
        return e;
    // start search of the admitted pairs; those with a hit join this
    // iteration's hot list, those that end here the finished list
    AlignParams S = srv->base;
    S.counters = b.d_cnt;
    S.easy_list = b.d_hot;
    S.hard_list = b.d_cold;
    S.list_in = srv->d_new;
    S.items_out = srv->d_items;
    if ((e = launch_search_items(S, NS, s))) return e;
    const uint64_t cap = srv->item_cap;
    S.list_slot = 0;
    S.items_in = srv->d_items;
    S.items_out = srv->d_items + cap;
    if ((e = launch_search(S, 16, 1, srv->search_blocks, s))) return e;
    S.items_in = srv->d_items + cap;
    S.items_out = srv->d_items;
    S.list_slot = 1;
    if ((e = launch_search(S, 16, 2, srv->search_blocks, s))) return e;
    S.items_in = srv->d_items;
    S.items_out = srv->d_items + cap;
    S.list_slot = 2;
    if ((e = launch_search(S, 16, 4, srv->search_blocks, s))) return e;
    if ((e = launch_search_finalize(S, NS, s))) return e;
    // windows until the iteration's deadline
    if ((e = launch_serve_stamp(b.d_params, srv->d_turn, s))) return e;
    AlignParams P = srv->base;
    P.counters = b.d_cnt;
    P.easy_list = b.d_hot;
    P.hard_list = b.d_cold;
    P.turn = srv->d_turn;
    P.arrivals = srv->d_arrivals;
    P.next_hot = nb.d_hot;
    P.next_cold = nb.d_cold;
    P.next_len = nb.d_cnt;
    if ((e = launch_windows(P, srv->win_blocks, s))) return e;
    return launch_serve_finish(srv->d_fin, srv->d_fin_len, srv->d_out, srv->d_fin_off, b.dh_hdr,
                               b.dh_slot, b.dh_res, srv->d_cigar, b.d_gather, srv->gather_cap, NS,
                               s);
}

void engine_main(genasm_server* srv);

}  // namespace

extern "C" {

uint64_t genasm_now_ns(void) { return steady_ns(); }

int genasm_server_create(genasm_ctx* ctx, const genasm_server_config* cfg_in,
                         genasm_server** out) {
    if (!ctx || !cfg_in || !out) return GENASM_E_INVAL;
    *out = nullptr;
    genasm_server_config cfg = *cfg_in;
    if (cfg.W < 2 || cfg.W > 64 || cfg.O < 0 || cfg.O >= cfg.W || cfg.k < 0) return GENASM_E_INVAL;
    if (cfg.max_slots == 0) cfg.max_slots = 32768;
    if (cfg.pool_bases == 0) cfg.pool_bases = 1ull << 29;
    if (cfg.max_pending == 0) cfg.max_pending = 65536;
    if (cfg.use_graph < 0 || cfg.use_graph > 1) cfg.use_graph = 1;
    if (cfg.iteration_us < 0 || cfg.iteration_us > 1000000) return GENASM_E_INVAL;
    if (cfg.cigar_runs < 0 || cfg.cigar_runs > 1) return GENASM_E_INVAL;
    if (cfg.max_slots > (1u << 24) || cfg.pool_bases > (1ull << 40)) return GENASM_E_INVAL;
    genasm_server* srv = new (std::nothrow) genasm_server();
    if (!srv) return GENASM_E_NOMEM;
    srv->ctx = ctx;
    srv->cfg = cfg;
    if (hipSetDevice(ctx->device) != hipSuccess) { delete srv; return GENASM_E_DEVICE; }
    const uint32_t NS = cfg.max_slots;
    const uint64_t pool_bytes = cfg.pool_bases / 4;
    const int L = cfg.W - cfg.O, stride = L + 2;
    const int lds_rows = 16;
    // window workgroups per CU: as many as stay resident together (the search
    // runs before the window kernel, not beside it)
    AlignParams occ{};
    occ.lds_rows = lds_rows;
    occ.stride = stride;
    occ.compact = 1;
    const int per_cu = std::max(1, std::min(16, windows_blocks_per_cu(occ)));
    srv->win_blocks = ctx->num_cus * per_cu;
    srv->groups = (uint32_t)srv->win_blocks * 4;
    srv->search_blocks = ctx->num_cus * 8;
    const uint64_t workers = (uint64_t)srv->win_blocks * 4;
    srv->upload_cap = 1ull << 24;
    srv->gather_cap = std::min<uint64_t>(cfg.pool_bases, 1ull << 23);

    bool ok = true;
    auto D = [&](auto*& p, size_t n) {
        using T = std::remove_reference_t<decltype(*p)>;
        p = dev_alloc<T>(n);
        ok = ok && p;
    };
    auto H = [&](auto*& p, size_t n) {
        using T = std::remove_reference_t<decltype(*p)>;
        p = host_alloc<T>(n);
        ok = ok && p;
    };
    // host memory the device writes: mapped, and its device address
    auto M = [&](auto*& h, auto*& d, size_t n) {
        using T = std::remove_reference_t<decltype(*h)>;
        h = host_alloc<T>(n, hipHostMallocMapped | hipHostMallocCoherent);
        void* dp = nullptr;
        ok = ok && h && hipHostGetDevicePointer(&dp, h, 0) == hipSuccess;
        d = static_cast<T*>(dp);
    };
    D(srv->d_pool, pool_bytes + 16);
    D(srv->d_plo, plane_words(cfg.pool_bases));
    D(srv->d_phi, plane_words(cfg.pool_bases));
    D(srv->d_cigar, cfg.pool_bases);  // a pair's CIGAR needs at most m + n elements
    D(srv->d_read_off, NS); D(srv->d_ref_off, NS); D(srv->d_run_base, NS);
    D(srv->d_read_len, NS); D(srv->d_ref_len, NS);
    D(srv->d_out, NS); D(srv->d_state, NS); D(srv->d_search, NS);
    D(srv->d_new, NS); D(srv->d_fin, NS); D(srv->d_fin_len, 4); D(srv->d_fin_off, NS);
    srv->item_cap = search_item_cap(NS, cfg.pool_bases, kServeSearchChunk);
    D(srv->d_items, 2 * srv->item_cap); D(srv->d_key, NS); D(srv->d_turn, 1);
    D(srv->d_arrivals, 1); H(srv->h_arrivals, 1);
    D(srv->d_spill, spill_words(workers, kCompactSpillRows));
    for (IterBufs& b : srv->it) {
        H(b.h_upload, srv->upload_cap); D(b.d_upload, srv->upload_cap);
        H(b.h_up_src, 2 * (size_t)NS); H(b.h_up_dst, 2 * (size_t)NS); H(b.h_up_word, 2 * (size_t)NS);
        H(b.h_up_len, 2 * (size_t)NS); H(b.h_up_bases, 2 * (size_t)NS);
        D(b.d_up_src, 2 * (size_t)NS); D(b.d_up_dst, 2 * (size_t)NS); D(b.d_up_word, 2 * (size_t)NS);
        D(b.d_up_len, 2 * (size_t)NS); D(b.d_up_bases, 2 * (size_t)NS);
        H(b.h_admit, NS); D(b.d_admit, NS);
        H(b.h_params, kServeParamWords); D(b.d_params, kServeParamWords);
        D(b.d_hot, NS); D(b.d_cold, NS); D(b.d_cnt, kCounterCount);
        M(b.h_hdr, b.dh_hdr, 2); M(b.h_slot, b.dh_slot, NS); M(b.h_res, b.dh_res, NS);
        D(b.d_gather, srv->gather_cap);
        ok = ok && hipEventCreate(&b.ev_start) == hipSuccess;
        ok = ok && hipEventCreate(&b.ev_done) == hipSuccess;
        ok = ok && hipEventCreateWithFlags(&b.ev_up, hipEventDisableTiming) == hipSuccess;
    }
    // pinned host blocks for submissions and completions, ready before the first request
    srv->hpool->warm(kArenaChunk, 32);
    srv->hpool->warm(8ull << 20, 2);
    srv->hpool->warm(16ull << 20, 2);
    ok = ok && hipStreamCreateWithFlags(&srv->s, hipStreamNonBlocking) == hipSuccess;
    ok = ok && hipStreamCreateWithFlags(&srv->s_copy, hipStreamNonBlocking) == hipSuccess;
    ok = ok && hipStreamCreateWithFlags(&srv->s_up, hipStreamNonBlocking) == hipSuccess;
    if (ok) {
        // both counters blocks start empty (no resident pairs)
        for (IterBufs& b : srv->it)
            ok = ok && hipMemsetAsync(b.d_cnt, 0, kCounterCount * sizeof(uint32_t), srv->s) == hipSuccess;
        ok = ok && hipStreamSynchronize(srv->s) == hipSuccess;
    }
    if (!ok) {
        (void)hipGetLastError();
        genasm_server_destroy(srv);
        return GENASM_E_NOMEM;
    }

    AlignParams& p = srv->base;
    p.reads = srv->d_pool;
    p.refs = srv->d_pool;
    p.read_lo = srv->d_plo;
    p.read_hi = srv->d_phi;
    p.ref_lo = srv->d_plo;
    p.ref_hi = srv->d_phi;
    p.planes_from_off0 = 0;
    p.read_off = srv->d_read_off;
    p.ref_off = srv->d_ref_off;
    p.read_len = srv->d_read_len;
    p.ref_len = srv->d_ref_len;
    p.run_base = srv->d_run_base;
    p.n_pairs = NS;
    p.K = std::min(cfg.k, cfg.W);
    p.W = cfg.W;
    p.L = L;
    p.stride = stride;
    p.out = srv->d_out;
    p.cigar = srv->d_cigar;
    p.cigar_cap = cfg.pool_bases;
    p.search = srv->d_search;
    p.spill = srv->d_spill;
    p.lds_rows = lds_rows;
    p.compact = 1;       // compact 16-lane window groups
    p.hard_row = 65;     // the search routes every pair with a hit to the hot list
    p.hard_lanes = 16;
    p.hard_share = 0;    // every worker drains the hot list before the cold one
    p.route = 1;
    p.state = srv->d_state;
    p.window_budget = cfg.window_budget;
    p.search_key = srv->d_key;
    p.search_chunk = kServeSearchChunk;
    p.fin_list = srv->d_fin;
    p.fin_len = srv->d_fin_len;

    if (cfg.use_graph) {
        for (int q = 0; q < 2; ++q) {
            IterBufs& b = srv->it[q];
            hipError_t e = hipStreamBeginCapture(srv->s, hipStreamCaptureModeThreadLocal);
            if (e == hipSuccess) {
                hipError_t e2 = enqueue_iteration(srv, q);
                e = hipStreamEndCapture(srv->s, &b.graph);
                if (e2 != hipSuccess) e = e2;
            }
            if (e == hipSuccess) e = hipGraphInstantiate(&b.exec, b.graph, nullptr, nullptr, 0);
            if (e != hipSuccess) {
                (void)hipGetLastError();
                genasm_server_destroy(srv);
                return GENASM_E_DEVICE;
            }
        }
    }
    srv->pool.reset(cfg.pool_bases);
    srv->cigpool.reset(cfg.pool_bases);
    srv->slots.resize(NS);
    srv->slot_tag.assign(NS, 0);
    srv->slot_state.assign(NS, 0);
    for (uint32_t i = NS; i-- > 0;) srv->free_slots.push_back(i);
    srv->engine = std::thread(engine_main, srv);
    *out = srv;
    return GENASM_OK;
}

}  // extern "C"

namespace {

// Checks one request's sizes against the server's pools.
// Room for `bytes` bytes of packed submissions in pinned memory: the tail of
// the current arena chunk, a new chunk, or (large submissions) a block of
// their own. False when no pinned memory can be had.
bool reserve_bytes(genasm_server* srv, uint64_t bytes, std::shared_ptr<uint8_t>* block, uint64_t* off) {
    bytes = std::max<uint64_t>(bytes, 1);
    if (bytes > kArenaChunk / 4) {
        *block = srv->hpool->get(bytes);
        *off = 0;
        return *block != nullptr;
    }
    std::lock_guard<std::mutex> lk(srv->arena_mu);
    if (!srv->arena || srv->arena_used + bytes > srv->arena_size) {
        srv->arena = srv->hpool->get(kArenaChunk);
        srv->arena_used = 0;
        srv->arena_size = srv->arena ? kArenaChunk : 0;
        if (!srv->arena) return false;
    }
    *block = srv->arena;
    *off = srv->arena_used;
    srv->arena_used += bytes;
    return true;
}

// Counts accepted requests (mu held) and, once per admission, copies the count
// to the device, where a running iteration's turns look for news (a turn may
// then end early and let the engine admit the new requests sooner). The copy
// runs on the copy stream beside the running kernels; if it cannot be queued
// the next submission tries again.
void note_arrivals(genasm_server* srv, uint64_t n) {
    srv->arrivals += n;
    *srv->h_arrivals = srv->arrivals;
    if (srv->signalled) return;
    int dev = -1;
    const bool switch_dev = hipGetDevice(&dev) != hipSuccess || dev != srv->ctx->device;
    if (switch_dev && hipSetDevice(srv->ctx->device) != hipSuccess) {
        (void)hipGetLastError();
        return;
    }
    if (hipMemcpyAsync(srv->d_arrivals, srv->h_arrivals, sizeof(unsigned long long),
                       hipMemcpyHostToDevice, srv->s_copy) == hipSuccess)
        srv->signalled = true;
    else
        (void)hipGetLastError();
    if (switch_dev && dev >= 0) (void)hipSetDevice(dev);
}

int check_request(const genasm_server* srv, uint64_t m, uint64_t n) {
    const uint64_t need = round_up(m, kBaseUnit) + round_up(n, kBaseUnit);
    if (m > 0x7fffffffull || n > 0x7fffffffull || need > srv->cfg.pool_bases ||
        (m + 3) / 4 + (n + 3) / 4 > srv->upload_cap || m + n + 1 > srv->cfg.pool_bases)
        return GENASM_E_TOOLONG;
    return GENASM_OK;
}

// Copies `nb` 2-bit bases starting at base `b0` of a packed stream to dst,
// starting at bit 0 of dst[0].
void copy_bases(uint8_t* dst, const uint8_t* src, uint64_t b0, uint64_t nb) {
    const uint64_t bytes = (nb + 3) / 4;
    const uint8_t* s = src + b0 / 4;
    const unsigned sh = (unsigned)(b0 % 4) * 2;
    if (sh == 0) {
        std::memcpy(dst, s, bytes);
    } else {
        // a byte takes its high part from the next source byte, which exists
        // for every byte but (possibly) the last: the range's last source byte
        // is `last - 1`, and no byte past it is read
        const uint64_t last = (b0 + nb + 3) / 4 - b0 / 4;  // source bytes the bases touch
        const uint64_t body = std::min(bytes, last - 1);
        for (uint64_t j = 0; j < body; ++j)
            dst[j] = (uint8_t)((s[j] >> sh) | ((unsigned)s[j + 1] << (8 - sh)));
        for (uint64_t j = body; j < bytes; ++j) dst[j] = (uint8_t)(s[j] >> sh);
    }
    // bases past nb in the last byte are zero
    if (nb % 4) dst[bytes - 1] &= (uint8_t)((1u << (2 * (nb % 4))) - 1);
}

}  // namespace

extern "C" {

int genasm_submit(genasm_server* srv, const char* read, uint64_t m, const char* ref, uint64_t n,
                  int32_t k, int32_t W, int32_t O, uint64_t tag) {
    if (!srv || (!read && m) || (!ref && n)) return GENASM_E_INVAL;
    if (k != srv->cfg.k || W != srv->cfg.W || O != srv->cfg.O) return GENASM_E_INVAL;
    int rc = check_request(srv, m, n);
    if (rc) return rc;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        if (srv->error) return srv->error;
        if (srv->pending.size() >= srv->cfg.max_pending) {
            srv->st.refused++;
            return GENASM_E_BUSY;
        }
    }
    Request r;
    const uint64_t rb = (m + 3) / 4;
    if (!reserve_bytes(srv, rb + (n + 3) / 4, &r.block, &r.off)) return GENASM_E_NOMEM;
    if (genasm_pack(read, m, r.block.get() + r.off, nullptr) != GENASM_OK ||
        genasm_pack(ref, n, r.block.get() + r.off + rb, nullptr) != GENASM_OK)
        return GENASM_E_ALPHABET;
    r.m = (uint32_t)m;
    r.n = (uint32_t)n;
    r.tag = tag;
    r.submit_ns = steady_ns();
    std::lock_guard<std::mutex> lk(srv->mu);
    if (srv->pending.size() >= srv->cfg.max_pending) {
        srv->st.refused++;
        return GENASM_E_BUSY;
    }
    srv->pending.push_back(std::move(r));
    srv->st.submitted++;
    srv->cv_work.notify_one();
    note_arrivals(srv, 1);
    return GENASM_OK;
}

int genasm_submit_batch(genasm_server* srv, const uint8_t* reads2b, const uint64_t* read_off,
                        const uint8_t* refs2b, const uint64_t* ref_off, uint64_t n_req,
                        int32_t k, int32_t W, int32_t O, const uint64_t* tags,
                        uint64_t* accepted) {
    if (!srv || !accepted) return GENASM_E_INVAL;
    *accepted = 0;
    if (n_req == 0) return GENASM_OK;
    if (!read_off || !ref_off || !tags) return GENASM_E_INVAL;
    if (k != srv->cfg.k || W != srv->cfg.W || O != srv->cfg.O) return GENASM_E_INVAL;
    for (uint64_t i = 0; i < n_req; ++i) {
        if (read_off[i + 1] < read_off[i] || ref_off[i + 1] < ref_off[i]) return GENASM_E_INVAL;
        int rc = check_request(srv, read_off[i + 1] - read_off[i], ref_off[i + 1] - ref_off[i]);
        if (rc) return rc;
    }
    if ((!reads2b && read_off[n_req] > read_off[0]) || (!refs2b && ref_off[n_req] > ref_off[0]))
        return GENASM_E_INVAL;
    uint64_t room;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        if (srv->error) return srv->error;
        room = srv->cfg.max_pending - std::min<uint64_t>(srv->pending.size(), srv->cfg.max_pending);
    }
    const uint64_t take = std::min(room, n_req);
    std::vector<Request> reqs(take);
    const uint64_t now = steady_ns();
    for (uint64_t i = 0; i < take; ++i) {
        Request& r = reqs[i];
        const uint64_t m = read_off[i + 1] - read_off[i], n = ref_off[i + 1] - ref_off[i];
        const uint64_t rb = (m + 3) / 4;
        if (!reserve_bytes(srv, rb + (n + 3) / 4, &r.block, &r.off)) return GENASM_E_NOMEM;
        if (m) copy_bases(r.block.get() + r.off, reads2b, read_off[i], m);
        if (n) copy_bases(r.block.get() + r.off + rb, refs2b, ref_off[i], n);
        r.m = (uint32_t)m;
        r.n = (uint32_t)n;
        r.tag = tags[i];
        r.submit_ns = now;
    }
    std::lock_guard<std::mutex> lk(srv->mu);
    for (Request& r : reqs) srv->pending.push_back(std::move(r));
    srv->st.submitted += take;
    *accepted = take;
    if (take < n_req) srv->st.refused += n_req - take;
    srv->cv_work.notify_one();
    note_arrivals(srv, take);
    return take < n_req ? GENASM_E_BUSY : GENASM_OK;
}

}  // extern "C"

namespace {

// Takes up to `max` finished records off the completion queue (waiting up to
// timeout_ms for the first), and no more than fit `runs_cap` elements when
// runs_cap is not ~0. Returns the count or a negative error; *first_need is
// set when not even the first record fits.
int take_done(genasm_server* srv, std::vector<DoneRec>& got, int max, uint64_t runs_cap,
              int timeout_ms, uint64_t* first_need) {
    std::unique_lock<std::mutex> lk(srv->mu);
    if (srv->done.empty() && timeout_ms > 0 && !srv->error)
        srv->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms),
                              [&] { return !srv->done.empty() || srv->error; });
    uint64_t used = 0;
    while ((int)got.size() < max && !srv->done.empty()) {
        const DoneRec& d = srv->done.front();
        if (runs_cap != ~0ull && used + d.result.cigar_len > runs_cap) {
            if (got.empty()) {
                *first_need = d.result.cigar_len;
                return GENASM_E_NOSPACE;
            }
            break;
        }
        used += d.result.cigar_len;
        got.push_back(std::move(srv->done.front()));
        srv->done.pop_front();
    }
    if (got.empty() && srv->error) return srv->error;
    return (int)got.size();
}

}  // namespace

extern "C" {

int genasm_poll(genasm_server* srv, genasm_completion* out, int max, int timeout_ms) {
    if (!srv || (!out && max > 0) || max < 0) return GENASM_E_INVAL;
    std::vector<DoneRec> got;
    uint64_t need = 0;
    const int k = take_done(srv, got, max, ~0ull, timeout_ms, &need);
    if (k < 0) return k;
    // the CIGAR, as text or as elements, copied here in the caller's thread
    static const char kOp[4] = {'=', 'X', 'I', 'D'};
    for (int i = 0; i < k; ++i) {
        const DoneRec& d = got[i];
        genasm_completion& c = out[i];
        c.tag = d.tag;
        c.result = d.result;
        c.result.cigar_off = 0;
        c.submit_ns = d.submit_ns;
        c.admit_ns = d.admit_ns;
        c.done_ns = d.done_ns;
        const uint32_t ne = d.result.cigar_len;
        const uint32_t* el = ne ? d.elements() : nullptr;
        if (srv->cfg.cigar_runs) {
            c.cigar = static_cast<char*>(std::malloc(std::max<size_t>(ne, 1) * 4));
            if (c.cigar && ne) std::memcpy(c.cigar, el, (size_t)ne * 4);
            if (!c.cigar) c.result.cigar_len = 0;
        } else {
            char* text = static_cast<char*>(std::malloc((size_t)ne * 11 + 1));
            char* w = text;
            if (text) {
                for (uint32_t e = 0; e < ne; ++e) {
                    char tmp[12];
                    int dg = 0;
                    uint32_t len = GENASM_CIGAR_LEN(el[e]);
                    do { tmp[dg++] = (char)('0' + len % 10); len /= 10; } while (len);
                    while (dg) *w++ = tmp[--dg];
                    *w++ = kOp[GENASM_CIGAR_OP(el[e])];
                }
                *w = '\0';
            }
            c.cigar = text;
            c.result.cigar_len = text ? (uint32_t)(w - text) : 0u;
        }
    }
    return k;
}

int genasm_poll_batch(genasm_server* srv, genasm_completion_info* out, int max, uint32_t* runs,
                      uint64_t runs_cap, uint64_t* runs_used, int timeout_ms) {
    if (!srv || !runs_used || max < 0 || (!out && max > 0) || (!runs && runs_cap)) return GENASM_E_INVAL;
    *runs_used = 0;
    std::vector<DoneRec> got;
    uint64_t need = 0;
    const int k = take_done(srv, got, max, runs_cap, timeout_ms, &need);
    if (k == GENASM_E_NOSPACE) *runs_used = need;
    if (k < 0) return k;
    uint64_t used = 0;
    for (int i = 0; i < k; ++i) {
        const DoneRec& d = got[i];
        genasm_completion_info& o = out[i];
        o.tag = d.tag;
        o.result = d.result;
        o.result.cigar_off = used;
        o.submit_ns = d.submit_ns;
        o.admit_ns = d.admit_ns;
        o.done_ns = d.done_ns;
        if (d.result.cigar_len)
            std::memcpy(runs + used, d.elements(), (size_t)d.result.cigar_len * 4);
        used += d.result.cigar_len;
    }
    *runs_used = used;
    return k;
}

void genasm_completion_release(genasm_completion* c) {
    if (c && c->cigar) {
        std::free(c->cigar);
        c->cigar = nullptr;
    }
}

int genasm_cancel(genasm_server* srv, uint64_t tag) {
    if (!srv) return GENASM_E_INVAL;
    std::lock_guard<std::mutex> lk(srv->mu);
    for (auto it = srv->pending.begin(); it != srv->pending.end(); ++it) {
        if (it->tag == tag) {
            srv->pending.erase(it);
            srv->st.cancelled++;
            return GENASM_OK;
        }
    }
    for (size_t slot = 0; slot < srv->slot_state.size(); ++slot) {
        if (srv->slot_state[slot] == 1 && srv->slot_tag[slot] == tag) {
            srv->slot_state[slot] = 2;
            srv->st.cancelled++;
            return GENASM_OK;
        }
    }
    return GENASM_E_INVAL;
}

int genasm_server_stats_read(genasm_server* srv, genasm_server_stats* out) {
    if (!srv || !out) return GENASM_E_INVAL;
    std::lock_guard<std::mutex> lk(srv->mu);
    *out = srv->st;
    out->pending = (uint32_t)srv->pending.size();
    return GENASM_OK;
}

void genasm_server_destroy(genasm_server* srv) {
    if (!srv) return;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stop = true;
        srv->cv_work.notify_all();
    }
    if (srv->engine.joinable()) srv->engine.join();
    (void)hipSetDevice(srv->ctx->device);
    if (srv->s) (void)hipStreamSynchronize(srv->s);
    if (srv->s_copy) (void)hipStreamSynchronize(srv->s_copy);
    if (srv->s_up) (void)hipStreamSynchronize(srv->s_up);
    std::vector<void*> dev = {srv->d_pool, srv->d_plo, srv->d_phi, srv->d_cigar, srv->d_read_off,
                              srv->d_ref_off, srv->d_run_base, srv->d_read_len, srv->d_ref_len,
                              srv->d_out, srv->d_state, srv->d_search, srv->d_new, srv->d_fin,
                              srv->d_fin_len, srv->d_fin_off, srv->d_items, srv->d_key,
                              srv->d_turn, srv->d_arrivals, srv->d_spill};
    std::vector<void*> host;
    for (IterBufs& b : srv->it) {
        if (b.exec) (void)hipGraphExecDestroy(b.exec);
        if (b.graph) (void)hipGraphDestroy(b.graph);
        for (void* p : {(void*)b.d_upload, (void*)b.d_up_src, (void*)b.d_up_dst, (void*)b.d_up_word,
                        (void*)b.d_up_len, (void*)b.d_up_bases, (void*)b.d_admit, (void*)b.d_params,
                        (void*)b.d_hot, (void*)b.d_cold, (void*)b.d_cnt, (void*)b.d_gather})
            dev.push_back(p);
        for (void* p : {(void*)b.h_upload, (void*)b.h_up_src, (void*)b.h_up_dst, (void*)b.h_up_word,
                        (void*)b.h_up_len, (void*)b.h_up_bases, (void*)b.h_admit, (void*)b.h_params,
                        (void*)b.h_hdr, (void*)b.h_slot, (void*)b.h_res})
            host.push_back(p);
        for (hipEvent_t e : {b.ev_start, b.ev_done, b.ev_up})
            if (e) (void)hipEventDestroy(e);
    }
    for (void* p : dev)
        if (p) (void)hipFree(p);
    for (void* p : host)
        if (p) (void)hipHostFree(p);
    if (srv->s) (void)hipStreamDestroy(srv->s);
    if (srv->s_copy) (void)hipStreamDestroy(srv->s_copy);
    if (srv->s_up) (void)hipStreamDestroy(srv->s_up);
    delete srv;
}

}  // extern "C"

namespace {

// Requests wait on the host, or at least half of the window groups hold a pair.
bool saturated(genasm_server* srv) {
    size_t pend;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        pend = srv->pending.size();
    }
    return pend > 0 || 2 * (uint64_t)srv->resident >= srv->groups;
}

// Admits waiting requests and queues iteration parity q on the device.
int launch_iteration(genasm_server* srv, int q) {
    RoctxRange range("genasm_serve_launch");
    IterBufs& b = srv->it[q];
    std::vector<Request> admitted;
    std::vector<uint32_t> admitted_slots;
    uint64_t admitted_arrivals = 0;
    {
        RoctxRange r_admit("genasm_serve_admit");
        std::lock_guard<std::mutex> lk(srv->mu);
        uint64_t upload = 0;
        const uint64_t now = steady_ns();
        while (!srv->pending.empty() && !srv->free_slots.empty()) {
            Request& r = srv->pending.front();
            const uint64_t bytes = r.bytes();
            if (upload + bytes > srv->upload_cap) break;
            uint64_t bs, cs;
            const uint64_t rl = round_up(r.m, kBaseUnit), fl = round_up(r.n, kBaseUnit);
            const uint64_t cl = (uint64_t)r.m + r.n + 1;
            uint32_t bh, ch;
            if (!srv->pool.alloc(rl + fl, &bh, &bs)) break;
            if (!srv->cigpool.alloc(cl, &ch, &cs)) {
                srv->pool.release(bh);
                break;
            }
            const uint32_t slot = srv->free_slots.back();
            srv->free_slots.pop_back();
            Slot& sl = srv->slots[slot];
            sl.tag = r.tag;
            sl.submit_ns = r.submit_ns;
            sl.admit_ns = now;
            sl.bstart = bs; sl.blen = rl + fl; sl.fstart = bs + rl; sl.cstart = cs; sl.clen = cl;
            sl.bh = bh;
            sl.ch = ch;
            srv->slot_tag[slot] = r.tag;
            srv->slot_state[slot] = 1;
            admitted_slots.push_back(slot);
            upload += bytes;
            admitted.push_back(std::move(r));
            srv->pending.pop_front();
        }
        srv->st.admitted += admitted.size();
        srv->st.pool_bases_used = srv->pool.used();
        // arrivals up to here are admitted (the queue is first in, first out);
        // later ones are news to this iteration's turns
        admitted_arrivals = srv->arrivals - srv->pending.size();
        srv->signalled = false;
    }
    // Uploads. Requests that lie back to back in one pinned submission block
    // form a run; a large run is copied to the device straight from its block,
    // a small one through the staging buffer (one copy for all of them). The
    // staged runs take the front of the device upload area, the direct ones
    // follow. Then the scatter ranges and admission records.
    RoctxRange r_stage("genasm_serve_stage");
    struct UpRun {
        const Request* first;
        uint64_t off, len, pos;
        bool direct;
    };
    std::vector<UpRun> upruns;
    std::vector<uint32_t> run_of(admitted.size());
    for (size_t a = 0; a < admitted.size(); ++a) {
        const Request& r = admitted[a];
        if (!upruns.empty() && upruns.back().first->block == r.block &&
            upruns.back().off + upruns.back().len == r.off) {
            upruns.back().len += r.bytes();
        } else {
            upruns.push_back(UpRun{&r, r.off, r.bytes(), 0, false});
        }
        run_of[a] = (uint32_t)(upruns.size() - 1);
    }
    constexpr uint64_t kDirectMin = 256ull << 10;
    uint64_t staged = 0;
    for (UpRun& u : upruns) {
        u.direct = u.len >= kDirectMin;
        if (!u.direct) {
            u.pos = staged;
            std::memcpy(b.h_upload + staged, u.first->block.get() + u.off, u.len);
            staged += u.len;
        }
    }
    uint64_t up = staged;
    for (UpRun& u : upruns) {
        if (u.direct) {
            u.pos = up;
            up += u.len;
        }
    }
    uint32_t nr = 0;
    for (size_t a = 0; a < admitted.size(); ++a) {
        const uint32_t slot = admitted_slots[a];
        const Slot& sl = srv->slots[slot];
        const Request& r = admitted[a];
        const UpRun& u = upruns[run_of[a]];
        const uint64_t at = u.pos + (r.off - u.off);  // the request's bytes in the upload area
        const uint64_t rb = r.read_bytes();
        const uint64_t part_off[2] = {0, rb};
        const uint64_t part_len[2] = {rb, r.bytes() - rb};
        const uint64_t dst[2] = {sl.bstart, sl.fstart};
        const uint32_t nb[2] = {r.m, r.n};
        for (int p = 0; p < 2; ++p) {
            if (part_len[p] == 0) continue;
            b.h_up_src[nr] = at + part_off[p];
            b.h_up_dst[nr] = dst[p] / 4;
            b.h_up_len[nr] = (uint32_t)part_len[p];
            b.h_up_word[nr] = dst[p] / 64;
            b.h_up_bases[nr] = nb[p];
            ++nr;
        }
        ServeAdmit& ad = b.h_admit[a];
        ad.read_off = sl.bstart;
        ad.ref_off = sl.fstart;
        ad.run_base = sl.cstart;
        ad.slot = slot;
        ad.m = r.m;
        ad.n = r.n;
        ad.pad = 0;
    }
    const uint32_t n_new = (uint32_t)admitted.size();
    srv->resident += n_new;
    b.n_new = n_new;
    // window time: 2 ms; while no request waits and most window groups are
    // free, a turn also ends from 250 us on once a pair of the iteration has
    // finished or a request has arrived (latency), else it runs the whole
    // window time (throughput). A configured window time is fixed.
    uint32_t us = (uint32_t)srv->cfg.iteration_us, soon_us = 0;
    if (us == 0) {
        us = 2000u;
        soon_us = saturated(srv) ? 0u : 250u;
    }
    b.h_params[kServeParamNew] = n_new;
    b.h_params[kServeParamTicks] = us * 100u;  // the device wall clock runs at 100 MHz
    b.h_params[kServeParamSoonTicks] = soon_us * 100u;
    b.h_params[kServeParamAdmitted] = (uint32_t)admitted_arrivals;
    b.h_params[kServeParamAdmitted + 1] = (uint32_t)(admitted_arrivals >> 32);
    // The uploads go on their own stream and overlap the running iteration (this
    // parity's buffers were last read by the iteration before it, which has
    // finished); the iteration waits for them on its stream.
    hipStream_t s = srv->s, su = srv->s_up;
    SRV_HIP(srv, hipEventRecord(b.ev_start, s));
    if (nr) {
        if (staged)
            SRV_HIP(srv, hipMemcpyAsync(b.d_upload, b.h_upload, staged, hipMemcpyHostToDevice, su));
        for (const UpRun& u : upruns) {
            if (!u.direct) continue;
            SRV_HIP(srv, hipMemcpyAsync(b.d_upload + u.pos, u.first->block.get() + u.off, u.len,
                                        hipMemcpyHostToDevice, su));
            b.holds.push_back(u.first->block);  // read by the copy until the iteration ends
        }
        SRV_HIP(srv, hipMemcpyAsync(b.d_up_src, b.h_up_src, nr * 8, hipMemcpyHostToDevice, su));
        SRV_HIP(srv, hipMemcpyAsync(b.d_up_dst, b.h_up_dst, nr * 8, hipMemcpyHostToDevice, su));
        SRV_HIP(srv, hipMemcpyAsync(b.d_up_len, b.h_up_len, nr * 4, hipMemcpyHostToDevice, su));
        SRV_HIP(srv, hipMemcpyAsync(b.d_up_word, b.h_up_word, nr * 8, hipMemcpyHostToDevice, su));
        SRV_HIP(srv, hipMemcpyAsync(b.d_up_bases, b.h_up_bases, nr * 4, hipMemcpyHostToDevice, su));
    }
    if (n_new)
        SRV_HIP(srv, hipMemcpyAsync(b.d_admit, b.h_admit, n_new * sizeof(ServeAdmit),
                                    hipMemcpyHostToDevice, su));
    SRV_HIP(srv, hipMemcpyAsync(b.d_params, b.h_params, kServeParamWords * 4, hipMemcpyHostToDevice, su));
    SRV_HIP(srv, hipEventRecord(b.ev_up, su));
    SRV_HIP(srv, hipStreamWaitEvent(s, b.ev_up, 0));
    if (nr) {
        SRV_HIP(srv, launch_scatter_bytes(b.d_upload, b.d_up_src, srv->d_pool, b.d_up_dst, b.d_up_len,
                                          nr, s));
        SRV_HIP(srv, launch_scatter_planes(b.d_upload, b.d_up_src, b.d_up_bases, srv->d_plo,
                                           srv->d_phi, b.d_up_word, nr, s));
    }
    if (b.exec) SRV_HIP(srv, hipGraphLaunch(b.exec, s));
    else SRV_HIP(srv, enqueue_iteration(srv, q));
    SRV_HIP(srv, hipEventRecord(b.ev_done, s));
    return GENASM_OK;
}

// Waits for iteration parity q and hands its finished pairs to the
// completion queue.
int finish_iteration(genasm_server* srv, int q) {
    RoctxRange range("genasm_serve_finish");
    IterBufs& b = srv->it[q];
    {
        RoctxRange r_wait("genasm_serve_wait");
        SRV_HIP(srv, hipEventSynchronize(b.ev_done));
    }
    b.holds.clear();  // the iteration's uploads are done
    float ms = 0.f;
    SRV_HIP(srv, hipEventElapsedTime(&ms, b.ev_start, b.ev_done));
    const uint32_t n_fin = (uint32_t)b.h_hdr[0];
    // the gathered elements that fit the buffer, in one copy into a pinned
    // block that the iteration's completions share; a pair past the buffer is
    // copied from the CIGAR pool by itself, to the end of the block
    uint64_t fit = 0, over_elems = 0;
    std::vector<uint32_t> over;
    for (uint32_t k = 0; k < n_fin; ++k) {
        const genasm_result& r = b.h_res[k];
        if (r.cigar_off + r.cigar_len <= srv->gather_cap) {
            fit = std::max(fit, r.cigar_off + r.cigar_len);
        } else {
            over.push_back(k);
            over_elems += r.cigar_len;
        }
    }
    std::shared_ptr<uint8_t> block;
    if (fit + over_elems) {
        block = srv->hpool->get((fit + over_elems) * 4);
        if (!block) return srv_fail(srv, "pinned completion block", hipErrorOutOfMemory);
    }
    uint32_t* els = reinterpret_cast<uint32_t*>(block.get());
    if (fit)
        SRV_HIP(srv, hipMemcpyAsync(els, b.d_gather, fit * 4, hipMemcpyDeviceToHost, srv->s_copy));
    uint64_t at = fit;
    std::vector<uint64_t> over_at(over.size());
    for (size_t j = 0; j < over.size(); ++j) {
        const uint32_t k = over[j];
        const Slot& sl = srv->slots[b.h_slot[k]];
        over_at[j] = at;
        SRV_HIP(srv, hipMemcpyAsync(els + at, srv->d_cigar + sl.cstart,
                                    (size_t)b.h_res[k].cigar_len * 4, hipMemcpyDeviceToHost,
                                    srv->s_copy));
        at += b.h_res[k].cigar_len;
    }
    SRV_HIP(srv, hipStreamSynchronize(srv->s_copy));
    RoctxRange r_records("genasm_serve_records");
    std::vector<DoneRec> recs(n_fin);
    size_t oj = 0;
    const uint64_t now = steady_ns();
    for (uint32_t k = 0; k < n_fin; ++k) {
        const uint32_t slot = b.h_slot[k];
        const Slot& sl = srv->slots[slot];
        DoneRec& d = recs[k];
        d.tag = sl.tag;
        d.result = b.h_res[k];
        if (oj < over.size() && over[oj] == k) d.result.cigar_off = over_at[oj++];
        d.submit_ns = sl.submit_ns;
        d.admit_ns = sl.admit_ns;
        d.done_ns = now;
        d.block = block;
        srv->pool.release(sl.bh);
        srv->cigpool.release(sl.ch);
    }
    srv->resident -= std::min(srv->resident, n_fin);
    std::lock_guard<std::mutex> lk(srv->mu);
    uint64_t delivered = 0;
    for (uint32_t k = 0; k < n_fin; ++k) {
        const uint32_t slot = b.h_slot[k];
        const bool cancelled = srv->slot_state[slot] == 2;
        srv->slot_state[slot] = 0;
        srv->free_slots.push_back(slot);
        if (cancelled) continue;  // cancelled while resident: no completion
        srv->done.push_back(std::move(recs[k]));
        ++delivered;
    }
    srv->st.completed += delivered;
    srv->st.iterations++;
    srv->st.device_ms += ms;
    srv->st.resident = srv->resident;
    srv->st.pool_bases_used = srv->pool.used();
    if (delivered) srv->cv_done.notify_all();
    return GENASM_OK;
}

void engine_main(genasm_server* srv) {
    if (hipSetDevice(srv->ctx->device) != hipSuccess) {
        srv_fail(srv, "hipSetDevice", hipErrorInvalidDevice);
        return;
    }
    std::deque<int> inflight;  // parities of the queued iterations, oldest first
    uint64_t t = 0;
    for (;;) {
        bool stop;
        size_t pend;
        {
            std::lock_guard<std::mutex> lk(srv->mu);
            stop = srv->stop;
            pend = srv->pending.size();
        }
        if (stop && inflight.empty()) return;
        const bool can_admit = pend > 0 && !srv->free_slots.empty();
        bool launch = false;
        // while work remains, a second iteration is queued behind the running
        // one, so that the device never waits for the host between them
        launch = !stop && inflight.size() < 2 && (can_admit || srv->resident > 0);
        if (launch) {
            const int q = (int)(t & 1);
            if (launch_iteration(srv, q) != GENASM_OK) return;
            inflight.push_back(q);
            ++t;
            continue;
        }
        if (!inflight.empty()) {
            const int q = inflight.front();
            inflight.pop_front();
            if (finish_iteration(srv, q) != GENASM_OK) return;
            continue;
        }
        std::unique_lock<std::mutex> lk(srv->mu);
        srv->cv_work.wait_for(lk, std::chrono::milliseconds(5),
                              [&] { return srv->stop || !srv->pending.empty(); });
    }
}

}  // namespace
