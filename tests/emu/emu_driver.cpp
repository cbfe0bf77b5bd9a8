// Host-side debugging driver: runs the unmodified GenASM kernels through the
// CPU emulation in tests/emu/hip/hip_runtime.h (plain or batched pipeline, or
// the device side of the serving loop).
//
//   emu_driver IN OUT
// IN : int64 form (0 plain, 1 batched, 2 serving loop, 3 unimproved, 4 filter), group_lanes, search_lanes,
//      lds_rows, k, W, O, n_pairs, read_bytes, ref_bytes, hard_row, window_budget,
//      slots, admit_per_iteration, hard_lanes, search_chunk, tb_prefetch, hard_share,
//      serving window time in emulated clock reads (0 = none), compact window groups (0/1);
//      then
//      the packed read bytes, the packed reference bytes, read_off[n+1], ref_off[n+1] (uint64).
// OUT: n genasm_result records, then (read bases + ref bases) CIGAR elements;
//      for the filter, n int32 distances then n uint32 starts.
#include "../../paper_2203_15561_amd/csrc/kernels.hip"

#include <algorithm>
#include <cstdio>
#include <numeric>
#include <vector>

namespace genasm { unsigned long long smem[kEmuLdsWords]; }

using namespace genasm;

static bool read_all(FILE* f, void* p, size_t n) { return n == 0 || fread(p, 1, n, f) == n; }

int main(int argc, char** argv) {
    if (argc != 3) { fprintf(stderr, "usage: emu_driver IN OUT\n"); return 2; }
    FILE* f = fopen(argv[1], "rb");
    if (!f) { perror("open IN"); return 2; }
    int64_t h[20];
    if (!read_all(f, h, sizeof h)) return 2;
    const int form = (int)h[0], G = (int)h[1], SG = (int)h[2], lds_rows = (int)h[3];
    const int k = (int)h[4], W = (int)h[5], O = (int)h[6];
    const uint64_t n = (uint64_t)h[7], nrb = (uint64_t)h[8], nfb = (uint64_t)h[9];
    const int hard_row = (int)h[10];
    const uint32_t budget = (uint32_t)h[11], n_slots = (uint32_t)h[12], per_iter = (uint32_t)h[13];
    const int hard_lanes = (int)h[14];
    const uint32_t chunk = (uint32_t)h[15];
    const int tb_prefetch = (int)h[16];
    const int hard_share = (int)h[17];
    const uint32_t ticks = (uint32_t)h[18];
    const int compact = (int)h[19];
    std::vector<uint8_t> reads(nrb + 8), refs(nfb + 8);
    std::vector<uint64_t> roff(n + 1), foff(n + 1);
    if (!read_all(f, reads.data(), nrb) || !read_all(f, refs.data(), nfb) ||
        !read_all(f, roff.data(), 8 * (n + 1)) || !read_all(f, foff.data(), 8 * (n + 1))) {
        fprintf(stderr, "short input\n");
        return 2;
    }
    fclose(f);
    reads.resize(nrb);  // exact sizes so that ASan sees reads past the end
    refs.resize(nfb);
    const uint64_t cap = (roff[n] - roff[0]) + (foff[n] - foff[0]);
    std::vector<genasm_result> out(n);
    std::vector<uint32_t> cigar(std::max<uint64_t>(cap, 1), 0xFFFFFFFFu);

    AlignParams p{};
    p.reads = reads.data();
    p.read_off = roff.data();
    p.refs = refs.data();
    p.ref_off = foff.data();
    p.n_pairs = n;
    p.K = std::min(k, W);
    p.W = W;
    p.L = W - O;
    p.stride = p.L + 2;
    p.out = out.data();
    p.cigar = cigar.data();
    p.cigar_cap = cap;
#if defined(GENASM_DEBUG)
    // debug build: per-pair audit words, handed to the results by the audit
    // kernel after the window work (plain and batched forms)
    std::vector<uint32_t> audit(std::max<uint64_t>(n, 1), 0u);
    p.audit = form == 2 ? nullptr : audit.data();
#endif
    // bit planes of both streams: from base 0 for the serving loop (slot offsets
    // are absolute), from the first offset otherwise, as the runtime does
    const bool serve = form == 2;
    const uint64_t rbases = serve ? roff[n] : roff[n] - roff[0];
    const uint64_t fbases = serve ? foff[n] : foff[n] - foff[0];
    std::vector<unsigned long long> rlo(plane_words(rbases)), rhi(plane_words(rbases));
    std::vector<unsigned long long> flo(plane_words(fbases)), fhi(plane_words(fbases));
    emu::group_lanes = 64;
    launch_planes(reads.data(), serve ? nullptr : roff.data(), rbases, rlo.data(), rhi.data(), nullptr);
    launch_planes(refs.data(), serve ? nullptr : foff.data(), fbases, flo.data(), fhi.data(), nullptr);
    p.read_lo = rlo.data();
    p.read_hi = rhi.data();
    p.ref_lo = flo.data();
    p.ref_hi = fhi.data();
    p.planes_from_off0 = serve ? 0 : 1;
    if (form == 4) {
        uint32_t max_m = 0;
        for (uint64_t i = 0; i < n; ++i) max_m = std::max<uint32_t>(max_m, (uint32_t)(roff[i + 1] - roff[i]));
        std::vector<int32_t> dist(n, -7);
        std::vector<uint32_t> start(n, 7u);
        emu::group_lanes = 64;
        if (launch_filter(reads.data(), roff.data(), refs.data(), foff.data(), n, max_m, k,
                          dist.data(), start.data(), nullptr) != hipSuccess) {
            fprintf(stderr, "filter launch rejected\n");
            return 3;
        }
        FILE* g = fopen(argv[2], "wb");
        if (!g) { perror("open OUT"); return 2; }
        fwrite(dist.data(), 4, n, g);
        fwrite(start.data(), 4, n, g);
        fclose(g);
        return 0;
    }
    if (form == 2) {
        // Serving loop, device side: slots are reused; each iteration admits
        // up to per_iter pairs into free slots (begin kernel), searches them,
        // then runs the window kernel over the two device lists until the
        // iteration's deadline (`ticks` reads of the emulated clock; 0 = none)
        // or `budget` windows per pair; the kernels move every pair to the
        // next iteration's lists or to the finished list.
        const int blocks = 2;
        const uint64_t workers = (uint64_t)blocks * 4;
        const int spill_rows = 64 - lds_rows;
        std::vector<SearchOut> search(n_slots, SearchOut{kSearchPending, 0});
        std::vector<uint32_t> cnt[2] = {std::vector<uint32_t>(kCounterCount, 0),
                                        std::vector<uint32_t>(kCounterCount, 0)};
        std::vector<uint32_t> hot[2] = {std::vector<uint32_t>(n_slots + 1), std::vector<uint32_t>(n_slots + 1)};
        std::vector<uint32_t> cold[2] = {std::vector<uint32_t>(n_slots + 1), std::vector<uint32_t>(n_slots + 1)};
        std::vector<uint32_t> params[2] = {std::vector<uint32_t>(kServeParamWords, 0),
                                           std::vector<uint32_t>(kServeParamWords, 0)};
        const uint64_t icap = search_item_cap(n_slots, foff[n], chunk);
        std::vector<uint64_t> items(2 * icap);
        std::vector<unsigned long long> key(n_slots);
        std::vector<uint32_t> new_list(n_slots + 1), fin(n_slots + 1), fin_len(1, 0);
        std::vector<ServeAdmit> admit(n_slots + 1);
        std::vector<unsigned long long> spill(spill_words(workers, kCompactSpillRows));
        std::vector<TurnLimits> turn(1);
        std::vector<unsigned long long> arrivals(1, 0);
        std::vector<uint64_t> s_roff(n_slots), s_foff(n_slots), s_base(n_slots);
        std::vector<uint32_t> s_rlen(n_slots), s_flen(n_slots);
        std::vector<PairState> state(n_slots);
        std::vector<genasm_result> s_out(n_slots);
        std::vector<int64_t> owner(n_slots, -1);
        std::vector<uint32_t> free_slots;
        for (uint32_t q = n_slots; q-- > 0;) free_slots.push_back(q);
        ServeSlots slots{s_roff.data(), s_foff.data(), s_base.data(), s_rlen.data(), s_flen.data(),
                         state.data()};
        p.read_off = s_roff.data();
        p.ref_off = s_foff.data();
        p.read_len = s_rlen.data();
        p.ref_len = s_flen.data();
        p.run_base = s_base.data();
        p.n_pairs = n_slots;
        p.out = s_out.data();
        p.search = search.data();
        p.spill = spill.data();
        p.lds_rows = lds_rows;
        p.compact = 1;
        p.hard_row = 65;
        p.hard_lanes = 16;
        p.hard_share = 0;
        p.route = 1;
        p.state = state.data();
        p.window_budget = budget;
        p.search_key = key.data();
        p.search_chunk = chunk;
        p.fin_list = fin.data();
        p.fin_len = fin_len.data();
        uint64_t next = 0, finished_n = 0, iters = 0, resident = 0;
        while (finished_n < n) {
            if (++iters > 100000) { fprintf(stderr, "serving loop does not finish\n"); return 3; }
            const int q = (int)(iters & 1);
            uint32_t n_new = 0;
            while (next < n && !free_slots.empty() && n_new < per_iter) {
                const uint32_t sl = free_slots.back();
                free_slots.pop_back();
                ServeAdmit& a = admit[n_new++];
                a.slot = sl;
                a.read_off = roff[next];
                a.m = (uint32_t)(roff[next + 1] - roff[next]);
                a.ref_off = foff[next];
                a.n = (uint32_t)(foff[next + 1] - foff[next]);
                a.run_base = (roff[next] - roff[0]) + (foff[next] - foff[0]);
                owner[sl] = (int64_t)next++;
                ++resident;
            }
            params[q][kServeParamNew] = n_new;
            // a turn may also end, from half the window time on, once a pair
            // of the iteration has finished
            params[q][kServeParamTicks] = ticks;
            params[q][kServeParamSoonTicks] = ticks / 2;
            emu::group_lanes = 64;
            launch_serve_begin(cnt[q].data(), cnt[1 - q].data(), fin_len.data(), params[q].data(),
                               admit.data(), slots, new_list.data(), nullptr);
            AlignParams S = p;
            S.counters = cnt[q].data();
            S.easy_list = hot[q].data();
            S.hard_list = cold[q].data();
            S.list_in = new_list.data();
            S.items_out = items.data();
            launch_search_items(S, n_slots, nullptr);
            emu::group_lanes = 16;
            S.list_slot = 0;
            S.items_in = items.data();
            S.items_out = items.data() + icap;
            launch_search(S, 16, 1, blocks, nullptr);
            S.items_in = items.data() + icap;
            S.items_out = items.data();
            S.list_slot = 1;
            launch_search(S, 16, 2, blocks, nullptr);
            S.items_in = items.data();
            S.items_out = items.data() + icap;
            S.list_slot = 2;
            launch_search(S, 16, 4, blocks, nullptr);
            emu::group_lanes = 64;
            launch_search_finalize(S, n_slots, nullptr);
            for (uint32_t i = 0; i < n_new; ++i) {
                if (search[admit[i].slot].row == kSearchPending) {
                    fprintf(stderr, "slot %u left pending by the search\n", admit[i].slot);
                    return 3;
                }
            }
            emu::group_lanes = 1;
            launch_serve_stamp(params[q].data(), turn.data(), nullptr);
            AlignParams P = p;
            P.counters = cnt[q].data();
            P.easy_list = hot[q].data();
            P.hard_list = cold[q].data();
            P.turn = turn.data();
            P.arrivals = arrivals.data();
            P.next_hot = hot[1 - q].data();
            P.next_cold = cold[1 - q].data();
            P.next_len = cnt[1 - q].data();
            emu::group_lanes = 16;
            launch_windows(P, blocks, nullptr);
            // the finished pairs' results (their CIGARs are already in place)
            for (uint32_t k = 0; k < fin_len[0]; ++k) {
                const uint32_t sl = fin[k];
                if (owner[sl] < 0 || !(state[sl].flags & kStateDone)) {
                    fprintf(stderr, "slot %u listed as finished but not done\n", sl);
                    return 3;
                }
                out[owner[sl]] = s_out[sl];
                owner[sl] = -1;
                free_slots.push_back(sl);
                ++finished_n;
                --resident;
            }
            // every resident pair is on exactly one of the next iteration's lists
            const uint32_t nh = cnt[1 - q][kCounterEasyLen], nc = cnt[1 - q][kCounterHardLen];
            if (nh + nc != resident) {
                fprintf(stderr, "lists hold %u + %u pairs, %llu resident\n", nh, nc,
                        (unsigned long long)resident);
                return 3;
            }
            std::vector<char> seen(n_slots, 0);
            for (uint32_t k = 0; k < nh + nc; ++k) {
                const uint32_t sl = k < nh ? hot[1 - q][k] : cold[1 - q][k - nh];
                if (sl >= n_slots || owner[sl] < 0 || seen[sl]++) {
                    fprintf(stderr, "bad list entry %u\n", sl);
                    return 3;
                }
            }
        }
        fprintf(stderr, "emu: serving loop finished in %llu iterations\n", (unsigned long long)iters);
    } else if (form == GENASM_FORM_PLAIN) {
        emu::group_lanes = 64;
        p.lds_rows = 64;
        launch_plain(p, nullptr);
        launch_audit(p, 0, nullptr);  // debug builds only
    } else if (form == GENASM_FORM_UNIMPROVED) {
        emu::group_lanes = 64;
        p.lds_rows = 64;
        std::vector<unsigned long long> table(unimproved_table_words(n));
        launch_unimproved(p, table.data(), nullptr);
    } else {
        const int blocks = 2;
        const uint64_t workers = (uint64_t)blocks * 4;
        const bool use_compact = compact && G == 16 && hard_lanes == 16;
        const int spill_rows = use_compact ? kCompactSpillRows : 64 - lds_rows;
        std::vector<SearchOut> search(n, SearchOut{kSearchPending, 0});
        std::vector<uint32_t> counters(kCounterCount, 0), order(n);
        const uint64_t icap = search_item_cap(n, foff[n] - foff[0], chunk);
        std::vector<uint64_t> items(2 * icap);
        std::vector<unsigned long long> key(n);
        std::vector<uint32_t> easy(n + 1), hard(n + 1);
        std::vector<unsigned long long> spill(spill_words(workers, spill_rows));
        std::iota(order.begin(), order.end(), 0u);
        std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) {
            return roff[a + 1] - roff[a] > roff[b + 1] - roff[b];
        });
        p.search = search.data();
        p.counters = counters.data();
        p.spill = spill_rows > 0 ? spill.data() : nullptr;
        p.order = order.data();
        p.easy_list = easy.data();
        p.hard_list = hard.data();
        p.hard_row = G == 64 ? 0 : hard_row;
        p.hard_lanes = G == 64 ? 64 : hard_lanes;
        p.tb_prefetch = tb_prefetch;
        p.hard_share = hard_share;
        p.route = 1;
        p.lds_rows = lds_rows;
        p.compact = use_compact ? 1 : 0;
        p.search_key = key.data();
        p.search_chunk = chunk;
        launch_init_counters(p.counters, (uint32_t)n, nullptr);
        p.list_in = p.order;
        p.items_out = items.data();
        emu::group_lanes = 64;
        launch_search_items(p, (uint32_t)n, nullptr);
        p.list_slot = 0;
        p.items_in = items.data();
        p.items_out = items.data() + icap;
        emu::group_lanes = SG;
        if (SG == 64) {
            launch_search(p, 64, 1, blocks, nullptr);
        } else {
            launch_search(p, 16, 1, blocks, nullptr);
            p.items_in = items.data() + icap;
            p.items_out = items.data();
            p.list_slot = 1;
            launch_search(p, 16, 2, blocks, nullptr);
            p.items_in = items.data();
            p.items_out = items.data() + icap;
            p.list_slot = 2;
            launch_search(p, 16, 4, blocks, nullptr);
        }
        emu::group_lanes = 64;
        launch_search_finalize(p, (uint32_t)n, nullptr);
        for (uint64_t i = 0; i < n; ++i) {
            if (search[i].row == kSearchPending) {
                fprintf(stderr, "pair %llu left pending by the search\n", (unsigned long long)i);
                return 3;
            }
        }
        p.list_in = nullptr;
        p.items_in = nullptr;
        p.items_out = nullptr;
        const uint32_t n_easy = counters[kCounterEasyLen], n_hard = counters[kCounterHardLen];
        if (p.hard_lanes != 16) {
            // The window kernel changes lane-group width between its two queues;
            // the emulation runs it once per queue with the matching group width.
            counters[kCounterEasyLen] = 0;
            emu::group_lanes = p.hard_lanes;
            launch_windows(p, blocks, nullptr);
            counters[kCounterEasyLen] = n_easy;
            counters[kCounterEasyHead] = 0;  // the first launch's easy loop popped past the end
            counters[kCounterHardLen] = 0;
            emu::group_lanes = 16;
            launch_windows(p, blocks, nullptr);
        } else {
            emu::group_lanes = 16;
            launch_windows(p, blocks, nullptr);
        }
        emu::group_lanes = 64;
        launch_audit(p, 1, nullptr);  // debug builds only
        fprintf(stderr, "emu: %u easy pairs, %u hard pairs\n", n_easy, n_hard);
    }
    FILE* g = fopen(argv[2], "wb");
    if (!g) { perror("open OUT"); return 2; }
    fwrite(out.data(), sizeof(genasm_result), n, g);
    fwrite(cigar.data(), 4, cigar.size(), g);
    fclose(g);
    return 0;
}
