// Randomized check of the serving pools' range allocator against a plain
// model of the allocated ranges: every range lies inside the pool and
// overlaps no other, the used count matches, a failure leaves no free gap of
// twice the request (plus the size-class rounding), and once everything is
// released the whole pool is one range again.
#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <iterator>
#include <map>
#include <random>

#include "range_alloc.h"

using genasm::RangeAlloc;

int main() {
    std::mt19937_64 g(7);
    for (int trial = 0; trial < 300; ++trial) {
        const uint64_t cap = 1 + g() % 5000;
        RangeAlloc A;
        A.reset(cap);
        std::map<uint64_t, std::pair<uint64_t, uint32_t>> live;  // start -> (length, handle)
        uint64_t used = 0;
        for (int op = 0; op < 2000; ++op) {
            if (live.empty() || g() % 2) {
                const uint64_t len = 1 + g() % (g() % 4 ? 40 : 800);
                uint32_t h;
                uint64_t st;
                if (A.alloc(len, &h, &st)) {
                    if (st + len > cap) return std::printf("range past the pool\n"), 1;
                    auto it = live.lower_bound(st);
                    if (it != live.end() && it->first < st + len) return std::printf("overlap\n"), 1;
                    if (it != live.begin() && std::prev(it)->first + std::prev(it)->second.first > st)
                        return std::printf("overlap\n"), 1;
                    live[st] = {len, h};
                    used += len;
                } else {
                    uint64_t prev = 0, gap = 0;
                    for (auto& kv : live) {
                        gap = std::max(gap, kv.first - prev);
                        prev = kv.first + kv.second.first;
                    }
                    gap = std::max(gap, cap - prev);
                    if (gap >= 2 * len + 16) return std::printf("failed with a gap of %llu for %llu\n",
                                                                (unsigned long long)gap,
                                                                (unsigned long long)len), 1;
                }
            } else {
                auto it = live.begin();
                std::advance(it, g() % live.size());
                A.release(it->second.second);
                used -= it->second.first;
                live.erase(it);
            }
            if (A.used() != used) return std::printf("used count differs\n"), 1;
        }
        for (auto& kv : live) A.release(kv.second.second);
        uint32_t h;
        uint64_t st;
        if (!A.alloc(cap, &h, &st) || st != 0) return std::printf("pool not whole again\n"), 1;
    }
    std::printf("ok\n");
    return 0;
}
