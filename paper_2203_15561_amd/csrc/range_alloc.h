// Range allocator of the serving engine's device pools (host-side bookkeeping,
// no device code): plain C++ so that it is tested on its own.
#pragma once

#include <cstdint>
#include <vector>

namespace genasm {

// Allocator of [0, cap) in abstract units with two-level segregated free
// lists: free ranges sit in lists by size class (the highest set bit, then
// the next kSl bits), with a bitmap of the non-empty lists, so that finding a
// range that fits, splitting it, and merging a released range with free
// neighbours are all constant time. A search starts at the class above the
// request's own (every range there fits) after a look at the first range of
// its own class, so it finds a good fit rather than the best one. Ranges are known by handle; their descriptors (start, size,
// neighbours by address, list links) live on the host, as the memory they
// describe is device memory.
class RangeAlloc {
  public:
    void reset(uint64_t cap) {
        d_.clear();
        spare_.clear();
        fl_map_ = 0;
        for (auto& m : sl_map_) m = 0;
        for (auto& h : head_)
            for (auto& x : h) x = kNone;
        used_ = 0;
        if (cap) {
            const uint32_t b = make({0, cap, kNone, kNone, kNone, kNone, true});
            link(b);
        }
    }
    // A range of `len` units (len >= 1): its handle and start, or false.
    bool alloc(uint64_t len, uint32_t* handle, uint64_t* start) {
        int fl, sl;
        // the first range of the request's own class, when it is long enough;
        // else any range of the classes above
        map_insert(len, &fl, &sl);
        uint32_t b = head_[fl][sl];
        if (b == kNone || d_[b].size < len) {
            map_search(len, &fl, &sl);
            if (fl >= kFl) return false;
            uint32_t sm = sl_map_[fl] & (~0u << sl);
            if (!sm) {
                const uint64_t fm = fl + 1 < 64 ? fl_map_ & (~0ull << (fl + 1)) : 0;
                if (!fm) return false;
                fl = __builtin_ctzll(fm);
                sm = sl_map_[fl];
            }
            sl = __builtin_ctz(sm);
            b = head_[fl][sl];
        }
        unlink(b);
        if (d_[b].size > len) {
            // the remainder becomes a free range of its own, next by address
            const uint32_t r = make({d_[b].start + len, d_[b].size - len, b, d_[b].next, kNone, kNone,
                                     true});
            if (d_[b].next != kNone) d_[d_[b].next].prev = r;
            d_[b].next = r;
            d_[b].size = len;
            link(r);
        }
        d_[b].free = false;
        used_ += len;
        *handle = b;
        *start = d_[b].start;
        return true;
    }
    void release(uint32_t b) {
        used_ -= d_[b].size;
        d_[b].free = true;
        const uint32_t nx = d_[b].next;
        if (nx != kNone && d_[nx].free) {
            unlink(nx);
            d_[b].size += d_[nx].size;
            d_[b].next = d_[nx].next;
            if (d_[b].next != kNone) d_[d_[b].next].prev = b;
            spare_.push_back(nx);
        }
        const uint32_t pv = d_[b].prev;
        if (pv != kNone && d_[pv].free) {
            unlink(pv);
            d_[pv].size += d_[b].size;
            d_[pv].next = d_[b].next;
            if (d_[pv].next != kNone) d_[d_[pv].next].prev = pv;
            spare_.push_back(b);
            b = pv;
        }
        link(b);
    }
    uint64_t used() const { return used_; }

  private:
    static constexpr int kSl = 4;   // second-level bits: 16 lists per power of two
    static constexpr int kFl = 61;  // first level: sizes below 16, then one per power of two
    static constexpr uint32_t kNone = ~0u;
    struct Desc {
        uint64_t start, size;
        uint32_t prev, next;      // neighbours by address
        uint32_t fprev, fnext;    // links in the free list of its class
        bool free;
    };
    static void map_insert(uint64_t size, int* fl, int* sl) {
        if (size < (1u << kSl)) {
            *fl = 0;
            *sl = (int)size;
            return;
        }
        const int m = 63 - __builtin_clzll(size);
        *fl = m - kSl + 1;
        *sl = (int)((size >> (m - kSl)) & ((1u << kSl) - 1));
    }
    // the class whose every range holds `size` units
    static void map_search(uint64_t size, int* fl, int* sl) {
        if (size >= (1u << kSl)) {
            const int m = 63 - __builtin_clzll(size);
            const uint64_t step = 1ull << (m - kSl);
            if (size > ~0ull - step) { *fl = kFl; *sl = 0; return; }
            size += step - 1;
        }
        map_insert(size, fl, sl);
    }
    uint32_t make(const Desc& d) {
        if (!spare_.empty()) {
            const uint32_t i = spare_.back();
            spare_.pop_back();
            d_[i] = d;
            return i;
        }
        d_.push_back(d);
        return (uint32_t)(d_.size() - 1);
    }
    void link(uint32_t b) {
        int fl, sl;
        map_insert(d_[b].size, &fl, &sl);
        d_[b].fprev = kNone;
        d_[b].fnext = head_[fl][sl];
        if (head_[fl][sl] != kNone) d_[head_[fl][sl]].fprev = b;
        head_[fl][sl] = b;
        fl_map_ |= 1ull << fl;
        sl_map_[fl] |= 1u << sl;
    }
    void unlink(uint32_t b) {
        int fl, sl;
        map_insert(d_[b].size, &fl, &sl);
        if (d_[b].fprev != kNone) d_[d_[b].fprev].fnext = d_[b].fnext;
        else head_[fl][sl] = d_[b].fnext;
        if (d_[b].fnext != kNone) d_[d_[b].fnext].fprev = d_[b].fprev;
        if (head_[fl][sl] == kNone) {
            sl_map_[fl] &= ~(1u << sl);
            if (!sl_map_[fl]) fl_map_ &= ~(1ull << fl);
        }
    }
    std::vector<Desc> d_;
    std::vector<uint32_t> spare_;
    uint64_t fl_map_ = 0;
    uint32_t sl_map_[kFl] = {};
    uint32_t head_[kFl][1 << kSl];
    uint64_t used_ = 0;
};

}  // namespace genasm
