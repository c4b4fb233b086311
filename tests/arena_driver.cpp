// Host-only randomized check of the request server's arena allocator.
#include <stdio.h>
#include <stdlib.h>

#include <map>
#include <random>

#include "arena.hpp"

int main(int argc, char **argv)
{
    const int seed = argc > 1 ? atoi(argv[1]) : 1;
    std::mt19937_64 rng(seed);
    const size_t size = (size_t)1 << 30;
    gpk::Arena a(size);
    std::map<size_t, size_t> live;   // off -> requested bytes
    size_t live_bytes = 0;
    for (int step = 0; step < 200000; ++step) {
        const bool do_alloc = live.empty() || (rng() % 100) < 55;
        if (do_alloc) {
            size_t n = 1 + rng() % ((rng() % 10 == 0) ? (size_t)200 << 20 : (size_t)4 << 20);
            size_t off;
            if (a.alloc(n, off)) {
                if (off % gpk::Arena::kAlign != 0) { printf("FAIL align\n"); return 1; }
                if (off + gpk::Arena::round(n) > size) { printf("FAIL bounds\n"); return 1; }
                auto nx = live.lower_bound(off);
                if (nx != live.end() && off + gpk::Arena::round(n) > nx->first) { printf("FAIL overlap next\n"); return 1; }
                if (nx != live.begin()) {
                    auto pv = std::prev(nx);
                    if (pv->first + gpk::Arena::round(pv->second) > off) { printf("FAIL overlap prev\n"); return 1; }
                }
                live[off] = n;
                live_bytes += gpk::Arena::round(n);
            } else if (a.largest_free() >= gpk::Arena::round(n)) {
                printf("FAIL refused although a block fits\n");
                return 1;
            }
        } else {
            auto it = live.begin();
            std::advance(it, rng() % live.size());
            a.release(it->first, it->second);
            live_bytes -= gpk::Arena::round(it->second);
            live.erase(it);
        }
        if (a.used() != live_bytes) { printf("FAIL used %zu vs %zu\n", a.used(), live_bytes); return 1; }
    }
    for (auto &kv : live) a.release(kv.first, kv.second);
    if (a.used() != 0 || a.free_blocks() != 1 || a.largest_free() != size) {
        printf("FAIL not coalesced: used %zu blocks %zu\n", a.used(), a.free_blocks());
        return 1;
    }
    printf("OK\n");
    return 0;
}
