// Serving form of the GenASM library: continuous batching of single-pair
// requests with device-resident sequences and per-pair window state.
//
// The engine thread runs device iterations. Each iteration admits waiting
// requests into free slots (bounded by the slot count, the base pool and the
// CIGAR pool), uploads their packed bases with one copy and one scatter
// kernel, then replays one captured graph:
//
//   init counters -> reset state of new slots -> { search stages on the new
//   slots } || { window kernel over the resident, already-searched slots,
//   each advancing at most window_budget windows }
//
// and finally returns the pairs that finished to the completion queue. A pair
// admitted in iteration t is searched in t and starts its windows in t+1, so a
// long start search never delays the window work of the pairs in flight.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "internal.h"

using namespace genasm;

namespace {

uint64_t steady_ns() {
    return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

// First-fit allocator of [0, cap) in abstract units.
class RangeAlloc {
  public:
    void reset(uint64_t cap) {
        free_.clear();
        if (cap) free_[0] = cap;
        used_ = 0;
    }
    bool alloc(uint64_t len, uint64_t* start) {
        if (len == 0) { *start = 0; return true; }
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= len) {
                *start = it->first;
                const uint64_t rest = it->second - len, s2 = it->first + len;
                free_.erase(it);
                if (rest) free_[s2] = rest;
                used_ += len;
                return true;
            }
        }
        return false;
    }
    void release(uint64_t start, uint64_t len) {
        if (len == 0) return;
        used_ -= len;
        auto it = free_.emplace(start, len).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    uint64_t used() const { return used_; }

  private:
    std::map<uint64_t, uint64_t> free_;
    uint64_t used_ = 0;
};

constexpr uint64_t kBaseUnit = 64;  // pool allocations in bases: whole bit-plane words

uint64_t round_up(uint64_t x, uint64_t a) { return (x + a - 1) / a * a; }

struct Request {
    std::vector<uint8_t> read2b, ref2b;
    uint32_t m = 0, n = 0;
    uint64_t tag = 0, submit_ns = 0;
};

struct Slot {
    bool busy = false;
    uint64_t tag = 0, submit_ns = 0, admit_ns = 0;
    uint64_t rstart = 0, rlen = 0, fstart = 0, flen = 0;  // pool ranges (bases)
    uint64_t cstart = 0, clen = 0;                        // CIGAR pool range (elements)
};

template <class T>
T* host_alloc(size_t n) {
    void* p = nullptr;
    if (hipHostMalloc(&p, std::max<size_t>(n, 1) * sizeof(T), hipHostMallocDefault) != hipSuccess)
        return nullptr;
    return static_cast<T*>(p);
}

template <class T>
T* dev_alloc(size_t n) {
    void* p = nullptr;
    if (hipMalloc(&p, std::max<size_t>(n, 1) * sizeof(T)) != hipSuccess) return nullptr;
    return static_cast<T*>(p);
}

}  // namespace

struct genasm_server {
    genasm_ctx* ctx = nullptr;
    genasm_server_config cfg{};
    AlignParams P{};      // window kernel parameters (fixed pointers)
    AlignParams S{};      // search parameters
    int search_blocks = 0, win_blocks = 0;
    hipStream_t s = nullptr, s2 = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr, ev_t0 = nullptr, ev_t1 = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;

    // device
    uint8_t* d_pool = nullptr;                 // 2-bit packed bases (start search)
    unsigned long long *d_plo = nullptr, *d_phi = nullptr;  // the same bases as bit planes (windows)
    uint32_t* d_cigar = nullptr;
    uint64_t *d_read_off = nullptr, *d_ref_off = nullptr, *d_run_base = nullptr;
    uint32_t *d_read_len = nullptr, *d_ref_len = nullptr;
    genasm_result* d_out = nullptr;
    PairState* d_state = nullptr;
    SearchOut* d_search = nullptr;
    uint32_t *d_counters = nullptr, *d_new = nullptr, *d_active = nullptr, *d_params = nullptr;
    uint64_t* d_items = nullptr;          // two start-search item lists
    unsigned long long* d_key = nullptr;  // per-slot search key
    uint64_t item_cap = 0;
    unsigned long long* d_spill = nullptr;
    uint8_t* d_upload = nullptr;
    uint64_t *d_up_src = nullptr, *d_up_dst = nullptr, *d_up_word = nullptr;
    uint32_t *d_up_len = nullptr, *d_up_bases = nullptr;
    uint32_t* d_gather_list = nullptr;
    uint64_t* d_gather_off = nullptr;
    uint32_t* d_gather = nullptr;
    uint64_t upload_cap = 0, gather_cap = 0;

    // pinned host mirrors
    uint64_t *h_read_off = nullptr, *h_ref_off = nullptr, *h_run_base = nullptr;
    uint32_t *h_read_len = nullptr, *h_ref_len = nullptr;
    uint32_t *h_new = nullptr, *h_active = nullptr, *h_params = nullptr;
    uint8_t* h_upload = nullptr;
    uint64_t *h_up_src = nullptr, *h_up_dst = nullptr, *h_up_word = nullptr;
    uint32_t *h_up_len = nullptr, *h_up_bases = nullptr;
    PairState* h_state = nullptr;
    genasm_result* h_out = nullptr;
    SearchOut* h_search = nullptr;
    uint32_t* h_gather_list = nullptr;
    uint64_t* h_gather_off = nullptr;
    uint32_t* h_gather = nullptr;

    // host state
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request> pending;
    std::deque<genasm_completion> done;
    std::vector<Slot> slots;
    std::vector<uint32_t> free_slots;
    std::vector<uint32_t> searched;  // resident, start search finished
    RangeAlloc pool, cigpool;
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

// The device work of one iteration: forked into the search chain (stream s)
// and the window kernel (stream s2). Used for graph capture and direct launch.
hipError_t enqueue_iteration(genasm_server* srv) {
    hipError_t e;
    const uint32_t n_slots = srv->cfg.max_slots;
    if ((e = launch_init_counters_dev(srv->d_counters, srv->d_params, srv->s))) return e;
    if ((e = launch_reset_states(srv->d_state, srv->d_new, srv->d_params, n_slots, srv->s))) return e;
    if ((e = hipEventRecord(srv->ev_fork, srv->s))) return e;
    if ((e = hipStreamWaitEvent(srv->s2, srv->ev_fork, 0))) return e;
    if ((e = launch_windows(srv->P, srv->win_blocks, srv->s2))) return e;
    if ((e = hipEventRecord(srv->ev_join, srv->s2))) return e;
    AlignParams S = srv->S;
    const uint64_t cap = srv->item_cap;
    S.list_in = srv->d_new;
    S.items_out = srv->d_items;
    if ((e = launch_search_items(S, n_slots, srv->s))) return e;
    S.list_slot = 0;
    S.items_in = srv->d_items;
    S.items_out = srv->d_items + cap;
    if ((e = launch_search(S, 16, 1, srv->search_blocks, srv->s))) return e;
    S.items_in = srv->d_items + cap;
    S.items_out = srv->d_items;
    S.list_slot = 1;
    if ((e = launch_search(S, 16, 2, srv->search_blocks, srv->s))) return e;
    S.items_in = srv->d_items;
    S.items_out = srv->d_items + cap;
    S.list_slot = 2;
    if ((e = launch_search(S, 16, 4, srv->search_blocks, srv->s))) return e;
    if ((e = launch_search_finalize(S, n_slots, srv->s))) return e;
    return hipStreamWaitEvent(srv->s, srv->ev_join, 0);
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
    if (cfg.max_slots == 0) cfg.max_slots = 8192;
    if (cfg.pool_bases == 0) cfg.pool_bases = 1ull << 28;
    if (cfg.max_pending == 0) cfg.max_pending = 65536;
    if (cfg.window_budget == 0) cfg.window_budget = 32;
    if (cfg.use_graph < 0 || cfg.use_graph > 1) cfg.use_graph = 1;
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
    // window workgroups per CU: one fewer than fit, leaving room for the start
    // search of newly admitted pairs, which runs beside the window kernel
    AlignParams occ{};
    occ.lds_rows = lds_rows;
    occ.stride = stride;
    const int per_cu = std::max(1, std::min(16, windows_blocks_per_cu(occ)) - 1);
    srv->win_blocks = ctx->num_cus * per_cu;
    srv->search_blocks = ctx->num_cus * 8;
    const uint64_t workers = (uint64_t)srv->win_blocks * 4;

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
    srv->upload_cap = 1ull << 24;
    srv->gather_cap = 1ull << 22;
    D(srv->d_pool, pool_bytes + 16);
    D(srv->d_plo, plane_words(cfg.pool_bases));
    D(srv->d_phi, plane_words(cfg.pool_bases));
    D(srv->d_cigar, cfg.pool_bases);  // a pair's CIGAR needs at most m + n elements
    D(srv->d_read_off, NS); D(srv->d_ref_off, NS); D(srv->d_run_base, NS);
    D(srv->d_read_len, NS); D(srv->d_ref_len, NS);
    D(srv->d_out, NS); D(srv->d_state, NS); D(srv->d_search, NS);
    srv->item_cap = search_item_cap(NS, cfg.pool_bases, kServeSearchChunk);
    D(srv->d_counters, kCounterCount); D(srv->d_items, 2 * srv->item_cap); D(srv->d_key, NS);
    D(srv->d_new, NS); D(srv->d_active, NS); D(srv->d_params, 4);
    D(srv->d_spill, spill_words(workers, 64 - lds_rows, stride));
    D(srv->d_upload, srv->upload_cap);
    D(srv->d_up_src, 2 * (size_t)NS); D(srv->d_up_dst, 2 * (size_t)NS); D(srv->d_up_len, 2 * (size_t)NS);
    D(srv->d_up_word, 2 * (size_t)NS); D(srv->d_up_bases, 2 * (size_t)NS);
    D(srv->d_gather_list, NS); D(srv->d_gather_off, NS); D(srv->d_gather, srv->gather_cap);
    H(srv->h_read_off, NS); H(srv->h_ref_off, NS); H(srv->h_run_base, NS);
    H(srv->h_read_len, NS); H(srv->h_ref_len, NS);
    H(srv->h_new, NS); H(srv->h_active, NS); H(srv->h_params, 4);
    H(srv->h_upload, srv->upload_cap);
    H(srv->h_up_src, 2 * (size_t)NS); H(srv->h_up_dst, 2 * (size_t)NS); H(srv->h_up_len, 2 * (size_t)NS);
    H(srv->h_up_word, 2 * (size_t)NS); H(srv->h_up_bases, 2 * (size_t)NS);
    H(srv->h_state, NS); H(srv->h_out, NS); H(srv->h_search, NS);
    H(srv->h_gather_list, NS); H(srv->h_gather_off, NS); H(srv->h_gather, srv->gather_cap);
    ok = ok && hipStreamCreateWithFlags(&srv->s, hipStreamNonBlocking) == hipSuccess;
    ok = ok && hipStreamCreateWithFlags(&srv->s2, hipStreamNonBlocking) == hipSuccess;
    ok = ok && hipEventCreateWithFlags(&srv->ev_fork, hipEventDisableTiming) == hipSuccess;
    ok = ok && hipEventCreateWithFlags(&srv->ev_join, hipEventDisableTiming) == hipSuccess;
    ok = ok && hipEventCreate(&srv->ev_t0) == hipSuccess;
    ok = ok && hipEventCreate(&srv->ev_t1) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        genasm_server_destroy(srv);
        return GENASM_E_NOMEM;
    }
    std::memset(srv->h_params, 0, 4 * sizeof(uint32_t));
    std::memset(srv->h_read_len, 0, NS * sizeof(uint32_t));
    std::memset(srv->h_ref_len, 0, NS * sizeof(uint32_t));
    std::memset(srv->h_read_off, 0, NS * sizeof(uint64_t));
    std::memset(srv->h_ref_off, 0, NS * sizeof(uint64_t));
    std::memset(srv->h_run_base, 0, NS * sizeof(uint64_t));

    AlignParams p{};
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
    p.counters = srv->d_counters;
    p.spill = srv->d_spill;
    p.lds_rows = lds_rows;
    p.hard_row = 65;
    p.hard_lanes = 16;
    p.hard_share = 100;
    p.route = 0;
    p.state = srv->d_state;
    p.window_budget = cfg.window_budget;
    p.search_key = srv->d_key;
    p.search_chunk = kServeSearchChunk;
    p.easy_list = srv->d_active;
    p.hard_list = srv->d_active;  // never used: the hard queue is empty
    srv->S = p;
    srv->P = p;

    if (cfg.use_graph) {
        hipError_t e = hipStreamBeginCapture(srv->s, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            hipError_t e2 = enqueue_iteration(srv);
            e = hipStreamEndCapture(srv->s, &srv->graph);
            if (e2 != hipSuccess) e = e2;
        }
        if (e == hipSuccess) e = hipGraphInstantiate(&srv->graph_exec, srv->graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            genasm_server_destroy(srv);
            return GENASM_E_DEVICE;
        }
    }
    srv->pool.reset(cfg.pool_bases);
    srv->cigpool.reset(cfg.pool_bases);
    srv->slots.resize(NS);
    for (uint32_t i = NS; i-- > 0;) srv->free_slots.push_back(i);
    srv->engine = std::thread(engine_main, srv);
    *out = srv;
    return GENASM_OK;
}

int genasm_submit(genasm_server* srv, const char* read, uint64_t m, const char* ref, uint64_t n,
                  int32_t k, int32_t W, int32_t O, uint64_t tag) {
    if (!srv || (!read && m) || (!ref && n)) return GENASM_E_INVAL;
    if (k != srv->cfg.k || W != srv->cfg.W || O != srv->cfg.O) return GENASM_E_INVAL;
    const uint64_t need = round_up(m, kBaseUnit) + round_up(n, kBaseUnit);
    if (m > 0x7fffffffull || n > 0x7fffffffull || need > srv->cfg.pool_bases ||
        need / 4 > srv->upload_cap || m + n + 1 > srv->cfg.pool_bases)
        return GENASM_E_TOOLONG;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        if (srv->error) return srv->error;
        if (srv->pending.size() >= srv->cfg.max_pending) {
            srv->st.refused++;
            return GENASM_E_BUSY;
        }
    }
    Request r;
    r.read2b.resize((m + 3) / 4);
    r.ref2b.resize((n + 3) / 4);
    if (genasm_pack(read, m, r.read2b.data(), nullptr) != GENASM_OK ||
        genasm_pack(ref, n, r.ref2b.data(), nullptr) != GENASM_OK)
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
    return GENASM_OK;
}

int genasm_poll(genasm_server* srv, genasm_completion* out, int max, int timeout_ms) {
    if (!srv || (!out && max > 0) || max < 0) return GENASM_E_INVAL;
    std::unique_lock<std::mutex> lk(srv->mu);
    if (srv->done.empty() && timeout_ms > 0 && !srv->error)
        srv->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms),
                              [&] { return !srv->done.empty() || srv->error; });
    int k = 0;
    while (k < max && !srv->done.empty()) {
        out[k++] = srv->done.front();
        srv->done.pop_front();
    }
    if (k == 0 && srv->error) return srv->error;
    return k;
}

void genasm_completion_release(genasm_completion* c) {
    if (c && c->cigar) {
        std::free(c->cigar);
        c->cigar = nullptr;
    }
}

int genasm_server_stats_read(genasm_server* srv, genasm_server_stats* out) {
    if (!srv || !out) return GENASM_E_INVAL;
    std::lock_guard<std::mutex> lk(srv->mu);
    *out = srv->st;
    out->pending = (uint32_t)srv->pending.size();
    out->pool_bases_used = srv->pool.used();
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
    if (srv->s2) (void)hipStreamSynchronize(srv->s2);
    for (auto& c : srv->done) genasm_completion_release(&c);
    if (srv->graph_exec) (void)hipGraphExecDestroy(srv->graph_exec);
    if (srv->graph) (void)hipGraphDestroy(srv->graph);
    void* dev[] = {srv->d_pool, srv->d_plo, srv->d_phi, srv->d_up_word, srv->d_up_bases, srv->d_cigar, srv->d_read_off, srv->d_ref_off, srv->d_run_base,
                   srv->d_read_len, srv->d_ref_len, srv->d_out, srv->d_state, srv->d_search,
                   srv->d_counters, srv->d_items, srv->d_key, srv->d_new, srv->d_active, srv->d_params,
                   srv->d_spill, srv->d_upload, srv->d_up_src, srv->d_up_dst, srv->d_up_len,
                   srv->d_gather_list, srv->d_gather_off, srv->d_gather};
    for (void* p : dev)
        if (p) (void)hipFree(p);
    void* host[] = {srv->h_up_word, srv->h_up_bases, srv->h_read_off, srv->h_ref_off, srv->h_run_base, srv->h_read_len,
                    srv->h_ref_len, srv->h_new, srv->h_active, srv->h_params, srv->h_upload,
                    srv->h_up_src, srv->h_up_dst, srv->h_up_len, srv->h_state, srv->h_out,
                    srv->h_search, srv->h_gather_list, srv->h_gather_off, srv->h_gather};
    for (void* p : host)
        if (p) (void)hipHostFree(p);
    for (hipEvent_t e : {srv->ev_fork, srv->ev_join, srv->ev_t0, srv->ev_t1})
        if (e) (void)hipEventDestroy(e);
    if (srv->s) (void)hipStreamDestroy(srv->s);
    if (srv->s2) (void)hipStreamDestroy(srv->s2);
    delete srv;
}

}  // extern "C"

namespace {

// One iteration; returns GENASM_OK or a device error (the engine then stops).
int iterate(genasm_server* srv, std::vector<uint32_t>& fresh) {
    const uint32_t NS = srv->cfg.max_slots;
    // 1. admission (FIFO) while a slot and room in both pools are free
    std::vector<Request> admitted;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        uint64_t upload = 0;
        while (!srv->pending.empty() && !srv->free_slots.empty()) {
            Request& r = srv->pending.front();
            const uint64_t bytes = r.read2b.size() + r.ref2b.size();
            if (!admitted.empty() && upload + bytes > srv->upload_cap) break;
            if (bytes > srv->upload_cap) break;  // cannot upload (pool check made at submit)
            uint64_t rs, fs, cs;
            const uint64_t rl = round_up(r.m, kBaseUnit), fl = round_up(r.n, kBaseUnit);
            const uint64_t cl = (uint64_t)r.m + r.n + 1;
            if (!srv->pool.alloc(rl, &rs)) break;
            if (!srv->pool.alloc(fl, &fs)) { srv->pool.release(rs, rl); break; }
            if (!srv->cigpool.alloc(cl, &cs)) {
                srv->pool.release(rs, rl);
                srv->pool.release(fs, fl);
                break;
            }
            const uint32_t slot = srv->free_slots.back();
            srv->free_slots.pop_back();
            Slot& sl = srv->slots[slot];
            sl.busy = true;
            sl.tag = r.tag;
            sl.submit_ns = r.submit_ns;
            sl.admit_ns = steady_ns();
            sl.rstart = rs; sl.rlen = rl; sl.fstart = fs; sl.flen = fl; sl.cstart = cs; sl.clen = cl;
            srv->h_read_off[slot] = rs;
            srv->h_read_len[slot] = r.m;
            srv->h_ref_off[slot] = fs;
            srv->h_ref_len[slot] = r.n;
            srv->h_run_base[slot] = cs;
            fresh.push_back(slot);
            upload += bytes;
            admitted.push_back(std::move(r));
            srv->pending.pop_front();
        }
        srv->st.admitted += admitted.size();
    }
    // 2. upload the admitted pairs' bases (one copy, one scatter) and the slot tables
    uint64_t up = 0;
    uint32_t nr = 0;
    for (size_t a = 0; a < admitted.size(); ++a) {
        const Slot& sl = srv->slots[fresh[fresh.size() - admitted.size() + a]];
        const Request& r = admitted[a];
        const std::vector<uint8_t>* parts[2] = {&r.read2b, &r.ref2b};
        const uint64_t dst[2] = {sl.rstart, sl.fstart};
        const uint32_t nb[2] = {r.m, r.n};
        for (int q = 0; q < 2; ++q) {
            if (parts[q]->empty()) continue;
            std::memcpy(srv->h_upload + up, parts[q]->data(), parts[q]->size());
            srv->h_up_src[nr] = up;
            srv->h_up_dst[nr] = dst[q] / 4;
            srv->h_up_len[nr] = (uint32_t)parts[q]->size();
            srv->h_up_word[nr] = dst[q] / 64;
            srv->h_up_bases[nr] = nb[q];
            up += parts[q]->size();
            ++nr;
        }
    }
    const uint32_t n_new = (uint32_t)fresh.size();
    const uint32_t n_act = (uint32_t)srv->searched.size();
    std::copy(fresh.begin(), fresh.end(), srv->h_new);
    std::copy(srv->searched.begin(), srv->searched.end(), srv->h_active);
    srv->h_params[0] = n_new;
    srv->h_params[1] = n_act;
    hipStream_t s = srv->s;
    SRV_HIP(srv, hipEventRecord(srv->ev_t0, s));
    if (nr) {
        SRV_HIP(srv, hipMemcpyAsync(srv->d_upload, srv->h_upload, up, hipMemcpyHostToDevice, s));
        SRV_HIP(srv, hipMemcpyAsync(srv->d_up_src, srv->h_up_src, nr * 8, hipMemcpyHostToDevice, s));
        SRV_HIP(srv, hipMemcpyAsync(srv->d_up_dst, srv->h_up_dst, nr * 8, hipMemcpyHostToDevice, s));
        SRV_HIP(srv, hipMemcpyAsync(srv->d_up_len, srv->h_up_len, nr * 4, hipMemcpyHostToDevice, s));
        SRV_HIP(srv, hipMemcpyAsync(srv->d_up_word, srv->h_up_word, nr * 8, hipMemcpyHostToDevice, s));
        SRV_HIP(srv, hipMemcpyAsync(srv->d_up_bases, srv->h_up_bases, nr * 4, hipMemcpyHostToDevice, s));
        SRV_HIP(srv, launch_scatter_bytes(srv->d_upload, srv->d_up_src, srv->d_pool, srv->d_up_dst,
                                          srv->d_up_len, nr, s));
        SRV_HIP(srv, launch_scatter_planes(srv->d_upload, srv->d_up_src, srv->d_up_bases,
                                           srv->d_plo, srv->d_phi, srv->d_up_word, nr, s));
    }
    if (n_new) {
        SRV_HIP(srv, hipMemcpyAsync(srv->d_read_off, srv->h_read_off, NS * 8, hipMemcpyHostToDevice, s));
        SRV_HIP(srv, hipMemcpyAsync(srv->d_ref_off, srv->h_ref_off, NS * 8, hipMemcpyHostToDevice, s));
        SRV_HIP(srv, hipMemcpyAsync(srv->d_run_base, srv->h_run_base, NS * 8, hipMemcpyHostToDevice, s));
        SRV_HIP(srv, hipMemcpyAsync(srv->d_read_len, srv->h_read_len, NS * 4, hipMemcpyHostToDevice, s));
        SRV_HIP(srv, hipMemcpyAsync(srv->d_ref_len, srv->h_ref_len, NS * 4, hipMemcpyHostToDevice, s));
        SRV_HIP(srv, hipMemcpyAsync(srv->d_new, srv->h_new, n_new * 4, hipMemcpyHostToDevice, s));
    }
    if (n_act)
        SRV_HIP(srv, hipMemcpyAsync(srv->d_active, srv->h_active, n_act * 4, hipMemcpyHostToDevice, s));
    SRV_HIP(srv, hipMemcpyAsync(srv->d_params, srv->h_params, 2 * 4, hipMemcpyHostToDevice, s));
    // 3. the device work of the iteration
    if (srv->graph_exec) SRV_HIP(srv, hipGraphLaunch(srv->graph_exec, s));
    else SRV_HIP(srv, enqueue_iteration(srv));
    SRV_HIP(srv, hipEventRecord(srv->ev_t1, s));
    // 4. which pairs finished: states of the searched pairs, search results of the new ones
    SRV_HIP(srv, hipMemcpyAsync(srv->h_state, srv->d_state, NS * sizeof(PairState),
                                hipMemcpyDeviceToHost, s));
    SRV_HIP(srv, hipMemcpyAsync(srv->h_out, srv->d_out, NS * sizeof(genasm_result),
                                hipMemcpyDeviceToHost, s));
    SRV_HIP(srv, hipStreamSynchronize(s));
    float ms = 0.f;
    SRV_HIP(srv, hipEventElapsedTime(&ms, srv->ev_t0, srv->ev_t1));
    std::vector<uint32_t> finished;
    std::vector<uint32_t> still;
    still.reserve(n_act + n_new);
    for (uint32_t i = 0; i < n_act; ++i) {
        const uint32_t slot = srv->h_active[i];
        (srv->h_state[slot].flags & kStateDone ? finished : still).push_back(slot);
    }
    for (uint32_t slot : fresh) {
        // a pair that ended in its start search (empty read, no hit) is done now
        (srv->h_state[slot].flags & kStateDone ? finished : still).push_back(slot);
    }
    srv->searched.swap(still);
    fresh.clear();
    // 5. CIGARs of the finished pairs: one gather kernel, one copy
    uint64_t total = 0;
    uint32_t ng = 0;
    for (uint32_t slot : finished) {
        srv->h_gather_list[ng] = slot;
        srv->h_gather_off[ng] = total;
        total += srv->h_out[slot].cigar_len;
        ++ng;
    }
    if (total > srv->gather_cap) {
        // grow the gather buffers
        SRV_HIP(srv, hipFree(srv->d_gather));
        SRV_HIP(srv, hipHostFree(srv->h_gather));
        srv->gather_cap = round_up(total, 1 << 20);
        srv->d_gather = dev_alloc<uint32_t>(srv->gather_cap);
        srv->h_gather = host_alloc<uint32_t>(srv->gather_cap);
        if (!srv->d_gather || !srv->h_gather) return srv_fail(srv, "gather buffer", hipErrorOutOfMemory);
    }
    if (total) {
        SRV_HIP(srv, hipMemcpyAsync(srv->d_gather_list, srv->h_gather_list, ng * 4, hipMemcpyHostToDevice, s));
        SRV_HIP(srv, hipMemcpyAsync(srv->d_gather_off, srv->h_gather_off, ng * 8, hipMemcpyHostToDevice, s));
        SRV_HIP(srv, launch_gather_runs(srv->d_out, srv->d_gather_list, ng, srv->d_gather_off,
                                        srv->d_cigar, srv->d_gather, s));
        SRV_HIP(srv, hipMemcpyAsync(srv->h_gather, srv->d_gather, total * 4, hipMemcpyDeviceToHost, s));
        SRV_HIP(srv, hipStreamSynchronize(s));
    }
    // 6. completions
    static const char kOp[4] = {'=', 'X', 'I', 'D'};
    std::vector<genasm_completion> comps(ng);
    for (uint32_t g = 0; g < ng; ++g) {
        const uint32_t slot = srv->h_gather_list[g];
        genasm_result r = srv->h_out[slot];
        std::string text;
        for (uint32_t e = 0; e < r.cigar_len; ++e) {
            const uint32_t el = srv->h_gather[srv->h_gather_off[g] + e];
            text += std::to_string(GENASM_CIGAR_LEN(el));
            text += kOp[GENASM_CIGAR_OP(el)];
        }
        genasm_completion& c = comps[g];
        c.tag = srv->slots[slot].tag;
        r.cigar_off = 0;
        r.cigar_len = (uint32_t)text.size();
        c.result = r;
        c.cigar = static_cast<char*>(std::malloc(text.size() + 1));
        if (c.cigar) std::memcpy(c.cigar, text.c_str(), text.size() + 1);
        c.submit_ns = srv->slots[slot].submit_ns;
        c.admit_ns = srv->slots[slot].admit_ns;
    }
    const uint64_t now = steady_ns();
    std::lock_guard<std::mutex> lk(srv->mu);
    for (uint32_t g = 0; g < ng; ++g) {
        const uint32_t slot = srv->h_gather_list[g];
        Slot& sl = srv->slots[slot];
        srv->pool.release(sl.rstart, sl.rlen);
        srv->pool.release(sl.fstart, sl.flen);
        srv->cigpool.release(sl.cstart, sl.clen);
        sl.busy = false;
        srv->free_slots.push_back(slot);
        comps[g].done_ns = now;
        srv->done.push_back(comps[g]);
    }
    srv->st.completed += ng;
    srv->st.iterations++;
    srv->st.device_ms += ms;
    srv->st.resident = (uint32_t)srv->searched.size();
    if (ng) srv->cv_done.notify_all();
    return GENASM_OK;
}

void engine_main(genasm_server* srv) {
    if (hipSetDevice(srv->ctx->device) != hipSuccess) {
        srv_fail(srv, "hipSetDevice", hipErrorInvalidDevice);
        return;
    }
    std::vector<uint32_t> fresh;
    for (;;) {
        {
            std::unique_lock<std::mutex> lk(srv->mu);
            if (srv->stop) return;
            if (srv->pending.empty() && srv->searched.empty()) {
                srv->cv_work.wait_for(lk, std::chrono::milliseconds(5));
                continue;
            }
        }
        if (iterate(srv, fresh) != GENASM_OK) return;
    }
}

}  // namespace
