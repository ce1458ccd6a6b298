// First-fit arena over offsets: the served engine's admission allocator,
// pure host logic with no HIP dependency (so that it can also be built on
// its own, e.g. under AddressSanitizer). Included by exactly one translation
// unit of the library (server.hip), which exports the bq_arena_* calls.
#pragma once
#include <stdint.h>

#include <iterator>
#include <map>
#include <new>

#include "bq.h"

struct bq_arena {
    uint64_t size, align, used, peak;
    std::map<uint64_t, uint64_t> free_blocks;  // offset -> length
    std::map<uint64_t, uint64_t> live;         // offset -> length
};

extern "C" {

bq_status bq_arena_create(uint64_t size, uint64_t align, bq_arena** out) {
    if (!out || size == 0 || align == 0 || (align & (align - 1))) return BQ_EINVAL;
    bq_arena* a = new (std::nothrow) bq_arena();
    if (!a) return BQ_ENOMEM;
    a->size = size & ~(align - 1);
    a->align = align;
    a->used = a->peak = 0;
    if (a->size) a->free_blocks[0] = a->size;
    *out = a;
    return BQ_OK;
}

bq_status bq_arena_destroy(bq_arena* a) {
    delete a;
    return BQ_OK;
}

bq_status bq_arena_alloc(bq_arena* a, uint64_t bytes, uint64_t* offset) {
    if (!a || !offset) return BQ_EINVAL;
    if (bytes == 0) bytes = 1;
    const uint64_t need = (bytes + a->align - 1) & ~(a->align - 1);
    for (auto it = a->free_blocks.begin(); it != a->free_blocks.end(); ++it) {
        if (it->second >= need) {
            const uint64_t off = it->first, len = it->second;
            a->free_blocks.erase(it);
            if (len > need) a->free_blocks[off + need] = len - need;
            a->live[off] = need;
            a->used += need;
            if (a->used > a->peak) a->peak = a->used;
            *offset = off;
            return BQ_OK;
        }
    }
    return BQ_EBUSY;
}

bq_status bq_arena_free(bq_arena* a, uint64_t offset) {
    if (!a) return BQ_EINVAL;
    auto it = a->live.find(offset);
    if (it == a->live.end()) return BQ_EINVAL;
    uint64_t off = it->first, len = it->second;
    a->live.erase(it);
    a->used -= len;
    // coalesce with the neighbours
    auto nx = a->free_blocks.lower_bound(off);
    if (nx != a->free_blocks.end() && nx->first == off + len) {
        len += nx->second;
        nx = a->free_blocks.erase(nx);
    }
    if (nx != a->free_blocks.begin()) {
        auto pv = std::prev(nx);
        if (pv->first + pv->second == off) {
            off = pv->first;
            len += pv->second;
            a->free_blocks.erase(pv);
        }
    }
    a->free_blocks[off] = len;
    return BQ_OK;
}

bq_status bq_arena_usage(const bq_arena* a, uint64_t* used, uint64_t* peak, uint64_t* largest_free) {
    if (!a) return BQ_EINVAL;
    if (used) *used = a->used;
    if (peak) *peak = a->peak;
    if (largest_free) {
        uint64_t best = 0;
        for (auto& kv : a->free_blocks) best = kv.second > best ? kv.second : best;
        *largest_free = best;
    }
    return BQ_OK;
}

}  // extern "C"

