// Device side of the Broker Queue (Section III.A, Alg. 1) for gfx950.
//
// The queue is a ring of N = 2^logN slots with one ticket per slot, a head
// and a tail position and a broker count. Alg. 1's protocol:
//  - ENSURE: an operation first reserves its right to run on `count`
//    (an enqueue only while count < N, a dequeue only while count > 0);
//    only reserved operations move head or tail.
//  - PUT_DATA / READ_DATA: position P is drawn from tail (head); slot P mod N
//    is used in round P / N; the enqueuer of round r waits for ticket 2r,
//    writes, and sets 2r+1; the dequeuer waits for 2r+1, reads, and sets
//    2(r+1), handing the slot to the next round's enqueuer.
//
// Wave64 form: a wavefront performs the operations of all its lanes as one.
// One lane reserves k slots on `count` with a single atomic, takes k
// consecutive positions from head/tail with a single atomic, and every lane
// derives its own position from the ballot of participating lanes and its
// rank among them (mbcnt). So a wave costs two contended atomics per batch
// instead of 2 per item. The per-slot ticket handshake stays per lane.
//
// Memory ordering: every queue word is accessed with agent-scope atomics
// (coherent across the separate L2s of the XCDs); ticket and payload share
// one word (see Queue), so the protocol needs no fences.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bq {

// ---------------------------------------------------------------------------
// control block: every hot word on its own 256-byte line
// ---------------------------------------------------------------------------
struct alignas(256) Word {
    unsigned long long v;
    unsigned long long pad[31];
};

enum : int {
    ERR_NONE = 0,
    ERR_TIMEOUT = 1,   // watchdog fired inside a wait
    ERR_RANGE = 2,     // key packing precondition failed
    ERR_FULL = 3,      // solver queue overflow (cannot happen by construction)
};

enum : int { ST_DEQ = 0, ST_RELAX, ST_PUSH, ST_FANOUT, ST_BATCH, ST_WALK, ST_SPIN, ST_IMPROVE, ST_IDLE, ST_POLL, ST_N };

struct Ctrl {
    Word head;       // next dequeue position (monotone)
    Word tail;       // next enqueue position (monotone)
    Word count;      // broker count (signed)
    Word pending;    // items enqueued or being processed (solver only)
    Word abort;      // != 0: every wave leaves its loop
    Word error;      // ERR_* of the first failure
    Word negcycle;   // solver: 1 when a negative cycle was proved
    Word aux[6];     // solver scratch: weight range, dequeue base and clock at start
    Word busy;       // solver with near / far buckets: near items taken, not yet retired
    Word stats[ST_N];
};

// ---------------------------------------------------------------------------
// wave helpers (every call site runs with the full wave active)
// ---------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ unsigned long long ballot(bool p) { return __ballot(p); }

// rank of this lane among the set bits of mask below it
__device__ __forceinline__ int rank_in(unsigned long long mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ uint32_t bcast32(uint32_t x) {
    return __builtin_amdgcn_readfirstlane(x);
}
__device__ __forceinline__ unsigned long long bcast64(unsigned long long x) {
    uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)x);
    uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(x >> 32));
    return ((unsigned long long)hi << 32) | lo;
}

// inclusive wave prefix sum of a 32-bit value (Hillis-Steele over wave64)
__device__ __forceinline__ int wave_incl_scan(int x) {
    // DPP, no LDS: lanes add the lane 1, 2, 4, 8 below them within their row
    // of 16 (lanes shifted in from outside the row read 0), then row 1 and 3
    // add the last lane of the row before, and rows 2 and 3 the last lane
    // of row 1
    x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, false);  // row_shr:1
    x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, false);  // row_shr:2
    x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, false);  // row_shr:4
    x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, false);  // row_shr:8
    x += __builtin_amdgcn_update_dpp(0, x, 0x142, 0xa, 0xf, false);  // row_bcast:15
    x += __builtin_amdgcn_update_dpp(0, x, 0x143, 0xc, 0xf, false);  // row_bcast:31
    return x;
}

// inclusive wave maximum scan of an unsigned value (same DPP steps; 0 is the
// identity)
__device__ __forceinline__ unsigned wave_incl_max(unsigned x) {
    unsigned y;
    y = (unsigned)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xf, 0xf, false);
    x = y > x ? y : x;
    y = (unsigned)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xf, 0xf, false);
    x = y > x ? y : x;
    y = (unsigned)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xf, 0xf, false);
    x = y > x ? y : x;
    y = (unsigned)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xf, 0xf, false);
    x = y > x ? y : x;
    y = (unsigned)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xa, 0xf, false);
    x = y > x ? y : x;
    y = (unsigned)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xc, 0xf, false);
    x = y > x ? y : x;
    return x;
}

// the value of the lane below (lane 0 reads 0): DPP wave_shr:1
__device__ __forceinline__ unsigned wave_shr1(unsigned x) {
    return (unsigned)__builtin_amdgcn_update_dpp(0, (int)x, 0x138, 0xf, 0xf, false);
}

// the value of lane 63
__device__ __forceinline__ int lane63(int x) { return __builtin_amdgcn_readlane(x, 63); }

// relaxed agent-scope atomics; P is a pointer in any address space
template <class P>
__device__ __forceinline__ auto ld_rlx(P p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class P, class V>
__device__ __forceinline__ void st_rlx(P p, V v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class P, class V>
__device__ __forceinline__ auto add_rlx(P p, V v) {
    return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void fence_acquire() { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent"); }
__device__ __forceinline__ void fence_release() { __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent"); }

// Alg. 1's sleep() inside WAIT_FOR_TICKET: a short s_sleep (64 clocks per
// unit) so spinning waves leave issue slots to the waves they wait for.
__device__ __forceinline__ void backoff(int level) {
    switch (level) {
        case 0: __builtin_amdgcn_s_sleep(1); break;
        case 1: __builtin_amdgcn_s_sleep(2); break;
        case 2: __builtin_amdgcn_s_sleep(8); break;
        default: __builtin_amdgcn_s_sleep(32); break;
    }
}

// Sleep of a wave that watches for work: doubles with `level` from one
// s_sleep unit (64 clocks) up to `max_units`. Callers size max_units to the
// number of watchers so that together they poll the hot lines at a bounded
// rate.
__device__ __forceinline__ void idle_backoff(int level, unsigned max_units) {
    unsigned units = level >= 20 ? max_units : (1u << level);
    if (units > max_units) units = max_units;
    while (units >= 127u) {
        __builtin_amdgcn_s_sleep(127);
        units -= 127u;
    }
    if (units >= 32u) __builtin_amdgcn_s_sleep(32);
    else if (units >= 8u) __builtin_amdgcn_s_sleep(8);
    else __builtin_amdgcn_s_sleep(1);
}

// 100 MHz constant clock (s_memrealtime)
__device__ __forceinline__ unsigned long long now_ticks() { return wall_clock64(); }

// ---------------------------------------------------------------------------
// queue view
//
// Slot layout (gfx950 form of Alg. 1's RingBuffer and Tickets): slot i is one
// 64-bit word, ticket in the high half and payload in the low half. The
// ticket handshake of PUT_DATA / READ_DATA then happens on a single word:
// the enqueuer that sees ticket 2r stores (2r+1, value) in one atomic store,
// the dequeuer that sees (2r+1, value) has the value in the same load and
// stores (2r+2, 0). Coherence of that one word orders everything, so no
// cross-XCD fence (L2 writeback / invalidate) is needed per operation.
// ---------------------------------------------------------------------------
// Device memory pointers kept in structures. In device code they are typed
// as global-memory pointers, so that accesses through a structure loaded
// from memory (the batched form's per-query descriptors) compile to global
// loads, stores and atomics rather than flat ones, which would also count
// against the LDS wait counter. Host code sees plain pointers and assigns
// them with a cast to the field's type.
#if defined(__HIP_DEVICE_COMPILE__)
#define BQ_GLOBAL __attribute__((address_space(1)))
#else
#define BQ_GLOBAL
#endif

struct Queue {
    BQ_GLOBAL unsigned long long* slots;  // [N] (ticket << 32 | payload)
    BQ_GLOBAL Ctrl* ctrl;                 // head, tail, count of this queue
    BQ_GLOBAL Ctrl* sig;                  // abort / error words (the same block, or
                                          // the first segment's for a segment of a
                                          // split queue)
    uint32_t logN;
    uint32_t pad;
    unsigned long long N;
};

__device__ __forceinline__ unsigned long long slot_word(uint32_t ticket, uint32_t val) {
    return ((unsigned long long)ticket << 32) | val;
}

// wave-uniform read of the abort word
__device__ __forceinline__ bool aborted(const Queue& q) {
    return bcast64(ld_rlx(&q.sig->abort.v)) != 0ull;
}

__device__ __forceinline__ void raise_error(const Queue& q, int code) {
    unsigned long long zero = 0ull;
    __hip_atomic_compare_exchange_strong(&q.sig->error.v, &zero, (unsigned long long)code,
                                         __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT);
    st_rlx(&q.sig->abort.v, 1ull);
}

// Watchdog: a wait that lasts longer than `limit` ticks (100 MHz) gives up.
struct Watch {
    unsigned long long start, limit;
    __device__ __forceinline__ void arm(unsigned long long lim) {
        limit = lim;
        start = now_ticks();
    }
    __device__ __forceinline__ bool expired() const { return now_ticks() - start > limit; }
};

// ENSURE for k enqueues (leader lane only): Alg. 1 ENSURE_ENQUEUE for a
// batch. Reserve k on count; the first min(k, N - old) are ensured, the rest
// are given back. Returns the number ensured.
__device__ __forceinline__ uint32_t reserve_enqueue(const Queue& q, uint32_t k) {
    BQ_GLOBAL long long* cnt = (BQ_GLOBAL long long*)(&q.ctrl->count.v);
    long long num = ld_rlx(cnt);
    if (num >= (long long)q.N) return 0;
    long long old = add_rlx(cnt, (long long)k);
    long long room = (long long)q.N - old;
    uint32_t e = room <= 0 ? 0u : (room >= (long long)k ? k : (uint32_t)room);
    if (e < k) add_rlx(cnt, -(long long)(k - e));
    return e;
}

// ENSURE for up to k dequeues (leader lane only), mirror image (reading of
// the dequeue broker: success when the count before the decrement was > 0).
// Asks only for what the count showed, so a crowd of idle waves does not
// drive the count far below zero.
// With `optimistic` (the caller's last reservation was full) the look at the
// count is skipped and k is asked for directly.
__device__ __forceinline__ uint32_t reserve_dequeue(const Queue& q, uint32_t k,
                                                    bool optimistic = false) {
    BQ_GLOBAL long long* cnt = (BQ_GLOBAL long long*)(&q.ctrl->count.v);
    if (!optimistic) {
        long long num = ld_rlx(cnt);
        if (num <= 0) return 0;
        if (num < (long long)k) k = (uint32_t)num;
    }
    long long old = add_rlx(cnt, -(long long)k);
    uint32_t e = old <= 0 ? 0u : (old >= (long long)k ? k : (uint32_t)old);
    if (e < k) add_rlx(cnt, (long long)(k - e));
    return e;
}

// Alg. 1 ENSURE_DEQUEUE as the solver runs it, under the two broker
// policies (leader lane only).
//  - Broker Queue: look at the count, take what it shows and, when a lost
//    race leaves the take empty while the count still shows items, look
//    again (the continuous re-validation; bounded here because the caller's
//    idle loop polls again anyway).
//  - BWD: a single take of k with no look before or after it: the count is
//    a snapshot, and a take that finds it short reports Empty.
__device__ __forceinline__ uint32_t ensure_dequeue(const Queue& q, uint32_t k, bool optimistic,
                                                   bool bwd) {
    if (bwd) return reserve_dequeue(q, k, true);
    uint32_t e = reserve_dequeue(q, k, optimistic);
    for (int again = 0; e == 0 && again < 3; ++again) {
        if (ld_rlx((BQ_GLOBAL long long*)(&q.ctrl->count.v)) <= 0) break;
        e = reserve_dequeue(q, k, false);
    }
    return e;
}

// Alg. 1 ENQUEUE's Full test and DEQUEUE's Empty test, read on 64-bit
// positions: Full when tail - head >= N, Empty when head >= tail.
__device__ __forceinline__ bool looks_full(const Queue& q) {
    unsigned long long h = ld_rlx(&q.ctrl->head.v), t = ld_rlx(&q.ctrl->tail.v);
    return (long long)(t - h) >= (long long)q.N;
}
__device__ __forceinline__ bool looks_empty(const Queue& q) {
    unsigned long long h = ld_rlx(&q.ctrl->head.v), t = ld_rlx(&q.ctrl->tail.v);
    return (long long)(t - h) <= 0;
}

// WAIT_FOR_TICKET for every active lane: poll the lane's slot word until its
// ticket half equals `want`; the word last read is returned in `word`. The
// whole wave loops together. Returns false on abort / watchdog.
__device__ __forceinline__ bool wait_slot(const Queue& q, bool active, unsigned long long pos,
                                          uint32_t want, unsigned long long& word,
                                          unsigned long long limit, unsigned long long& spins) {
    const unsigned long long* p = &q.slots[pos & (q.N - 1ull)];
    Watch wd;
    wd.arm(limit);
    int level = 0;
    for (uint32_t it = 0;; ++it) {
        bool ready = true;
        if (active) {
            word = ld_rlx(p);
            ready = (uint32_t)(word >> 32) == want;
        }
        if (__all(ready)) return true;
        ++spins;
        if ((it & 63u) == 63u) {
            if (aborted(q)) return false;
            if (wd.expired()) {
                if (lane_id() == 0) raise_error(q, ERR_TIMEOUT);
                return false;
            }
            if (level < 3) ++level;
        }
        backoff(level);
    }
}

__device__ __forceinline__ uint32_t round_of(const Queue& q, unsigned long long pos) {
    return (uint32_t)(pos >> q.logN);
}

// PUT_DATA for active lanes at their positions: wait for ticket 2r, store
// (2r+1, value).
__device__ __forceinline__ bool put_slots(const Queue& q, bool active, unsigned long long pos,
                                          uint32_t val, unsigned long long limit,
                                          unsigned long long& spins) {
    const uint32_t r = round_of(q, pos);
    unsigned long long w = 0;
    if (!wait_slot(q, active, pos, 2u * r, w, limit, spins)) return false;
    if (active) st_rlx(&q.slots[pos & (q.N - 1ull)], slot_word(2u * r + 1u, val));
    return true;
}

// READ_DATA: wait for (2r+1, value), take the value, hand the slot to round
// r+1 by storing (2(r+1), 0).
__device__ __forceinline__ bool read_slots(const Queue& q, bool active, unsigned long long pos,
                                           uint32_t& val, unsigned long long limit,
                                           unsigned long long& spins) {
    const uint32_t r = round_of(q, pos);
    unsigned long long w = 0;
    if (!wait_slot(q, active, pos, 2u * r + 1u, w, limit, spins)) return false;
    if (active) {
        val = (uint32_t)w;
        st_rlx(&q.slots[pos & (q.N - 1ull)], slot_word(2u * (r + 1u), 0u));
    }
    return true;
}

}  // namespace bq
