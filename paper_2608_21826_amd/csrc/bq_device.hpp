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
// Memory ordering: slot and ticket accesses use agent-scope atomics; a wave
// that saw its tickets runs one agent-scope acquire fence before touching
// the slots, and one agent-scope release fence before publishing tickets.
// On a multi-XCD gfx950 agent these fences are what makes data written by a
// wave on one XCD visible to a wave on another (separate L2s).
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
};

enum : int { ST_DEQ = 0, ST_RELAX, ST_PUSH, ST_FANOUT, ST_BATCH, ST_WALK, ST_SPIN, ST_IMPROVE, ST_N };

struct Ctrl {
    Word head;       // next dequeue position (monotone)
    Word tail;       // next enqueue position (monotone)
    Word count;      // broker count (signed)
    Word pending;    // items enqueued or being processed (solver only)
    Word abort;      // != 0: every wave leaves its loop
    Word error;      // ERR_* of the first failure
    Word negcycle;   // solver: 1 when a negative cycle was proved
    Word aux[6];     // solver scratch: weight range, dequeue base and clock at start
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
    const int l = lane_id();
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        int y = __shfl_up(x, off, 64);
        if (l >= off) x += y;
    }
    return x;
}

template <class T>
__device__ __forceinline__ T ld_rlx(const T* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T>
__device__ __forceinline__ void st_rlx(T* p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T>
__device__ __forceinline__ T add_rlx(T* p, T v) {
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

// Longer sleeps for waves that found no work: up to ~16 us between polls so
// thousands of idle waves do not flood the count/pending lines.
__device__ __forceinline__ void idle_backoff(int level) {
    if (level < 4) {
        backoff(level);
        return;
    }
    const int reps = 1 << (level - 4);  // 1..8 x 127 units of 64 clocks
    for (int i = 0; i < reps; ++i) __builtin_amdgcn_s_sleep(127);
}

// 100 MHz constant clock (s_memrealtime)
__device__ __forceinline__ unsigned long long now_ticks() { return wall_clock64(); }

// ---------------------------------------------------------------------------
// queue view
// ---------------------------------------------------------------------------
struct Queue {
    uint32_t* tickets;   // [N]
    uint32_t* ring;      // [N]
    Ctrl* ctrl;
    uint32_t logN;
    uint32_t pad;
    unsigned long long N;
};

// wave-uniform read of the abort word
__device__ __forceinline__ bool aborted(const Queue& q) {
    return bcast64(ld_rlx(&q.ctrl->abort.v)) != 0ull;
}

__device__ __forceinline__ void raise_error(const Queue& q, int code) {
    unsigned long long zero = 0ull;
    __hip_atomic_compare_exchange_strong(&q.ctrl->error.v, &zero, (unsigned long long)code,
                                         __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT);
    st_rlx(&q.ctrl->abort.v, 1ull);
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
    long long* cnt = reinterpret_cast<long long*>(&q.ctrl->count.v);
    long long num = ld_rlx(cnt);
    if (num >= (long long)q.N) return 0;
    long long old = add_rlx(cnt, (long long)k);
    long long room = (long long)q.N - old;
    uint32_t e = room <= 0 ? 0u : (room >= (long long)k ? k : (uint32_t)room);
    if (e < k) add_rlx(cnt, -(long long)(k - e));
    return e;
}

// ENSURE for k dequeues (leader lane only), mirror image (reading of the
// dequeue broker: success when the count before the decrement was > 0).
__device__ __forceinline__ uint32_t reserve_dequeue(const Queue& q, uint32_t k) {
    long long* cnt = reinterpret_cast<long long*>(&q.ctrl->count.v);
    long long num = ld_rlx(cnt);
    if (num <= 0) return 0;
    long long old = add_rlx(cnt, -(long long)k);
    uint32_t e = old <= 0 ? 0u : (old >= (long long)k ? k : (uint32_t)old);
    if (e < k) add_rlx(cnt, (long long)(k - e));
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

// Wait until every active lane's slot carries its expected ticket. Whole
// wave loops together. Returns false on abort/timeout.
__device__ __forceinline__ bool wait_tickets(const Queue& q, bool active, uint32_t slot,
                                             uint32_t want, unsigned long long limit,
                                             unsigned long long& spins) {
    Watch wd;
    wd.arm(limit);
    int level = 0;
    for (uint32_t it = 0;; ++it) {
        bool ready = !active || ld_rlx(&q.tickets[slot]) == want;
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

// PUT_DATA for lanes with `active`: positions base + rank. Values are written
// after the acquire fence that follows the ticket wait and published by
// release fence + ticket store.
__device__ __forceinline__ bool put_slots(const Queue& q, bool active, unsigned long long pos,
                                          uint32_t val, unsigned long long limit,
                                          unsigned long long& spins) {
    const uint32_t slot = (uint32_t)(pos & (q.N - 1));
    const uint32_t round = (uint32_t)(pos >> q.logN);
    if (!wait_tickets(q, active, slot, 2u * round, limit, spins)) return false;
    fence_acquire();
    if (active) st_rlx(&q.ring[slot], val);
    fence_release();
    if (active) st_rlx(&q.tickets[slot], 2u * round + 1u);
    return true;
}

// READ_DATA: wait for 2r+1, read, hand the slot to round r+1 with 2(r+1).
__device__ __forceinline__ bool read_slots(const Queue& q, bool active, unsigned long long pos,
                                           uint32_t& val, unsigned long long limit,
                                           unsigned long long& spins) {
    const uint32_t slot = (uint32_t)(pos & (q.N - 1));
    const uint32_t round = (uint32_t)(pos >> q.logN);
    if (!wait_tickets(q, active, slot, 2u * round + 1u, limit, spins)) return false;
    fence_acquire();
    if (active) val = ld_rlx(&q.ring[slot]);
    fence_release();
    if (active) st_rlx(&q.tickets[slot], 2u * (round + 1u));
    return true;
}

}  // namespace bq
