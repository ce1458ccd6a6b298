// Host-only check of the served engine's arena (arena_host.hpp), built on
// its own under AddressSanitizer and UndefinedBehaviorSanitizer by
// tests/test_sanitizers.py. Random alloc / free sequences are checked
// against an independent model over the live blocks: every offset is
// aligned, inside the arena and disjoint from the other live blocks; an
// allocation is the first gap (in address order) that is large enough, and
// fails only when no gap is; used / peak / largest free match the model.
// Exit status 0 when every check holds.
#include <stdio.h>
#include <stdlib.h>

#include <algorithm>
#include <map>
#include <random>
#include <vector>

#include "arena_host.hpp"

static int fail(const char* what, unsigned long long a, unsigned long long b) {
    fprintf(stderr, "arena check failed: %s (%llu, %llu)\n", what, a, b);
    return 1;
}

// gaps between live blocks over [0, size): (offset, length), address order
static std::vector<std::pair<uint64_t, uint64_t>> gaps(const std::map<uint64_t, uint64_t>& live,
                                                       uint64_t size) {
    std::vector<std::pair<uint64_t, uint64_t>> g;
    uint64_t at = 0;
    for (auto& kv : live) {
        if (kv.first > at) g.push_back({at, kv.first - at});
        at = kv.first + kv.second;
    }
    if (size > at) g.push_back({at, size - at});
    return g;
}

static int run(uint64_t size, uint64_t align, unsigned seed, int ops) {
    bq_arena* a = nullptr;
    if (bq_arena_create(size, align, &a) != BQ_OK) return fail("create", size, align);
    const uint64_t usable = size & ~(align - 1);
    std::mt19937_64 rng(seed);
    std::map<uint64_t, uint64_t> live;  // model: offset -> rounded length
    uint64_t peak = 0;
    for (int i = 0; i < ops; ++i) {
        const bool do_alloc = live.empty() || (rng() % 100) < 55;
        if (do_alloc) {
            uint64_t bytes = rng() % (usable / 6 + 2);
            if (rng() % 8 == 0) bytes = rng() % (2 * align + 1);
            const uint64_t need = ((bytes ? bytes : 1) + align - 1) & ~(align - 1);
            uint64_t off = ~0ull;
            const bq_status st = bq_arena_alloc(a, bytes, &off);
            uint64_t expect = ~0ull;
            for (auto& gp : gaps(live, usable))
                if (gp.second >= need) {
                    expect = gp.first;
                    break;
                }
            if (expect == ~0ull) {
                if (st != BQ_EBUSY) return fail("alloc succeeded without a fitting gap", need, off);
                continue;
            }
            if (st != BQ_OK) return fail("alloc refused with a fitting gap", need, expect);
            if (off != expect) return fail("not first fit", off, expect);
            if (off % align) return fail("misaligned", off, align);
            if (off + need > usable) return fail("past the end", off, need);
            live[off] = need;
        } else {
            auto it = live.begin();
            std::advance(it, (long)(rng() % live.size()));
            if (bq_arena_free(a, it->first) != BQ_OK) return fail("free", it->first, 0);
            live.erase(it);
            if (bq_arena_free(a, usable + align) != BQ_EINVAL) return fail("bad free", 0, 0);
        }
        uint64_t used_m = 0;
        for (auto& kv : live) used_m += kv.second;
        peak = std::max(peak, used_m);
        uint64_t largest_m = 0;
        for (auto& gp : gaps(live, usable)) largest_m = std::max(largest_m, gp.second);
        uint64_t used = 0, pk = 0, largest = 0;
        bq_arena_usage(a, &used, &pk, &largest);
        if (used != used_m) return fail("used", used, used_m);
        if (pk != peak) return fail("peak", pk, peak);
        if (largest != largest_m) return fail("largest free", largest, largest_m);
    }
    for (auto& kv : live) bq_arena_free(a, kv.first);
    uint64_t used = 1, largest = 0;
    bq_arena_usage(a, &used, nullptr, &largest);
    if (used != 0 || largest != usable) return fail("not whole after freeing all", used, largest);
    bq_arena_destroy(a);
    return 0;
}

int main() {
    const uint64_t sizes[] = {1ull << 12, (1ull << 16) + 300, 1ull << 30, 4096 * 7 + 17};
    const uint64_t aligns[] = {1, 64, 256, 4096};
    unsigned seed = 1;
    for (uint64_t sz : sizes)
        for (uint64_t al : aligns) {
            if (al > sz) continue;
            if (run(sz, al, seed++, 3000)) return 1;
        }
    bq_arena* a = nullptr;
    if (bq_arena_create(100, 3, &a) != BQ_EINVAL) return fail("odd align accepted", 0, 0);
    printf("arena ok\n");
    return 0;
}
