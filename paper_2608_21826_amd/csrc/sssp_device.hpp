// Device side of the queue-driven Bellman-Ford solver (shared by the
// single-query and batched launches), for the queue-based Bellman-Ford of
// Section III.C driven by the Broker Queue of Section III.A.
//
// Work item: a vertex u whose distance dropped. A wave dequeues up to 64*b
// items with one ticket, stages them in LDS with their edge ranges, scans the
// concatenated CSR rows with all 64 lanes (coalesced reads of cols/w), lowers
// each target with a 64-bit atomicMin (Alg. 3's relax rule: a source at
// infinity never relaxes; a target is lowered when source + weight is
// smaller) and enqueues every target whose distance dropped and that was not
// already queued.
//
// One 64-bit key per vertex carries everything the relax needs, so each
// step is a single atomic on a single word:
//
//      key = d << S | parent << 1 | q        (S = PB + 1, PB = bits for n)
//
//  - d: the current distance label (signed); parent: the vertex whose edge
//    set it (all ones = none); q: 1 while the vertex has an item in the queue.
//  - relax u->v: atomicMin(key[v], (d_u + w) << S | u << 1 | 1). Signed order
//    of keys is the order of (d, parent, q). If the minimum took our value,
//    v's label dropped (or kept its distance with a smaller parent); if the
//    old q was 0 this lane now owes one enqueue of v; if it was 1 the item
//    already in the queue will read the new label.
//  - dequeue of u: atomicAnd(key[u], ~1) clears q and returns the label in
//    the same atomic, so no relax can slip between the two.
//  - the final key gives d and, as parent, the smallest-id in-neighbour u
//    with d(u) + w(u,v) = d(v): every such u relaxes v with its final label
//    at least once, and the minimum keeps the smallest.
//
// High-degree rows are split: a vertex with more than C = 2^chunk_log edges
// scans only the part of its row inside its first global chunk
// [jC, (j+1)C) and enqueues the later chunks of its row as items n + j, which
// other waves take (chunk_owner[j] = u names the vertex).
//
// Queue segments (the paper's partitioned queue of Section III.B, applied
// to the chip's XCDs instead of to GPUs): the solver may split its queue
// into up to 8 Broker Queues, each with its own ring, head, tail and count
// on separate lines. Workgroups are dispatched to the XCDs in turn, so
// workgroup i calls segment i mod nseg home: its waves publish there and
// dequeue there first, and take from the fullest other queue when their own
// are empty. Each hot word then carries 1/nseg of the traffic. Every queue
// can hold all items, so no enqueue ever finds one Full.
//
// Chunk lane: each home segment s also has a second Broker Queue (queue
// nseg + s) for the row chunks its waves publish. A chunk item is part of
// the scan of a vertex already dequeued, not new work, so a wave takes from
// its chunk queue before its vertex queue: a hub's row is then scanned
// right after the hub's dequeue, as the method's "dequeue u, scan u's row"
// reads, instead of behind everything enqueued meanwhile. On RMAT-20 this
// cut the solve from 2.85 to 2.64 ms at the same launch. Improved vertices
// whose rows are longer than one chunk go there too: most labels improve
// through the hubs, so scanning them early saves rescans elsewhere (RMAT-20
// about 5 % faster at the same launch). The row length costs one load per
// published vertex, so a wave starts routing only once it has met a long
// row (a graph without any, like a road mesh, never pays for it). Each lane
// stays FIFO.
//
// Termination: the global counter `pending` equals the live items
// (published and not yet fully processed) plus every wave's debt: the items
// a wave retired without subtracting them yet. A wave pays a publish of k
// items out of its debt when it can and adds only the rest to pending, and
// gives its whole debt back before it waits for work. The counter is raised
// before items become visible, so it is 0 only when no item is live and no
// wave holds debt: then the work is done. While the queue is busy most
// batches publish about as much as they retire, so pending sees few atomics.
//
// Negative cycles (Alg. 3 detects them as changes in round n-1; a queue has
// no rounds): (1) a label below (n-1) * min(0, min w) is impossible without
// one; (2) once the dequeued work exceeds a few times n, some waves walk the
// parent pointers (Brent's cycle finding); a closed walk of real edges whose
// weights sum below zero proves a negative cycle reachable from src.
// Marking mode (minus infinity) does not stop there: a candidate below the
// bound, or the vertex a walk found on a negative cycle, takes the key
// KEY_NEG, which is below every label. A dequeued minus-infinity vertex
// hands every out-neighbour a candidate below the bound, so the mark spreads
// through the queue like any lowered label, over exactly the vertices that a
// negative cycle reaches. When the queue empties, every reachable negative
// cycle holds a marked vertex (otherwise its edges would all be satisfied
// and their slacks, which sum to the cycle's weight, could not be negative),
// and the unmarked labels are exact.
#pragma once
#include <hip/hip_runtime.h>
#include <limits.h>

#include "bq_device.hpp"

namespace {

using bq::Queue;

constexpr long long KEY_INF = 0x7FFFFFFFFFFFFFFELL;  // d = max, parent = all ones, q = 0
// minus infinity (marking mode): below every packed label; q = 1 while queued
constexpr long long KEY_NEG = LLONG_MIN | 1ll;

__device__ __forceinline__ bool is_neg_key(long long k) { return k <= KEY_NEG; }
constexpr int SOLVE_WG = 256;                 // batched solver workgroup
constexpr int WAVES_PER_WG = SOLVE_WG / 64;
// single-query solver workgroup: two waves, so that the few hundred waves a
// query can feed spread over every CU (and its vector-memory pipeline)
// instead of filling half of them
constexpr int SOLVE_WG_ONE = 128;
constexpr int WAVES_PER_WG_ONE = SOLVE_WG_ONE / 64;
constexpr int OUTCAP = 1024;  // LDS push buffer per wave
#ifndef SSSP_UNROLL
#define SSSP_UNROLL 8
#endif
// waves per SIMD the solver kernels are compiled for (register budget:
// 512 / SSSP_MIN_WAVES per lane)
#ifndef SSSP_MIN_WAVES
#define SSSP_MIN_WAVES 2
#endif
constexpr int U = SSSP_UNROLL;  // edges per lane per pipelined step
// near / far buckets: far work is taken only while at most this many near
// items per wave of the grid are in flight (half a batch): waiting for none
// leaves most waves idle, never waiting lets the far queues run ahead
constexpr unsigned long long FAR_GATE_PER_WAVE = 32;

struct SolveArgs {
    Queue q;
    BQ_GLOBAL const long long* off;
    BQ_GLOBAL const int* col;
    BQ_GLOBAL const int* w;
    BQ_GLOBAL long long* key;  // the caller's dist buffer, used as key array
    BQ_GLOBAL unsigned* chunk_owner;  // [m >> chunk_log + 1]
    BQ_GLOBAL const int* wrange;  // per-block (min w, max w) from k_init
    int n;
    int src;
    long long m;
    unsigned shift;          // S = PB + 1
    unsigned chunk_log;
    unsigned long long limit;     // one wait (ticks of the 100 MHz clock)
    unsigned long long deadline;  // whole solve
    BQ_GLOBAL unsigned long long* trace;  // optional timeline: 4 words per sample
    unsigned trace_shift;         // one sample per 2^trace_shift dequeued items
    unsigned trace_cap;           // samples
    unsigned bwd;                 // dequeue broker policy: 0 Broker Queue, 1 BWD
    unsigned nseg;                // queue segments, 1..MAX_SEG; queue s < nq
                                  // (s < nseg: vertex queue of home s; s < 2 nseg:
                                  // chunk queue of home s - nseg; s < 3 nseg: far
                                  // queue of home s - 2 nseg) has slots
                                  // q.slots + s * q.N, control q.ctrl + s
    unsigned nq;                  // queues in use: 2 nseg, or 3 nseg with buckets
    long long bucket_width;       // 0: one FIFO per home; k > 0: near / far split at
                                  // a threshold T that advances in steps of
                                  // k * max(1, max |w|) / 16 (see solve_instance)
    unsigned neginf;              // 1: mark minus infinity instead of stopping
    unsigned fan_bulk;            // 1: a row's chunk items are published with one
                                  // reservation per OUTCAP items (the batched
                                  // form); 0: 64 at a time (one query: publishing
                                  // a hub's chunks faster gets its row scanned
                                  // before the labels it spreads have settled,
                                  // k 2.50 -> 2.64 on RMAT-20)
    // Key layout. Null: vertex v's key is key[v] and queue items are vertex
    // ids. Otherwise (the batched form's degree-class layout of a shared
    // graph) keys and vertex items are key positions: key position t holds
    // the key of original vertex orig[t] = v and pos[v] = t. Row offsets and
    // the parent field of a key stay in original ids; the edges of each row
    // are read from tcol (target key positions) and tw (weights), in which
    // every row is reordered by the class of its targets.
    BQ_GLOBAL const unsigned* tcol;
    BQ_GLOBAL const int* tw;
    BQ_GLOBAL const unsigned* orig;
    BQ_GLOBAL const unsigned* pos;
};

// original vertex of key position t, and key position of original vertex v
__device__ __forceinline__ unsigned orig_of(const SolveArgs& a, unsigned t) {
    return a.orig ? a.orig[t] : t;
}
__device__ __forceinline__ unsigned pos_of(const SolveArgs& a, unsigned v) {
    return a.pos ? a.pos[v] : v;
}
// key position of edge e's target, and its weight
__device__ __forceinline__ int target_of(const SolveArgs& a, long long e) {
    return a.tcol ? (int)a.tcol[e] : a.col[e];
}
__device__ __forceinline__ int weight_of(const SolveArgs& a, long long e) {
    return a.tw ? a.tw[e] : a.w[e];
}

constexpr unsigned MAX_SEG = 8;             // gfx950: one segment per XCD
constexpr unsigned MAX_Q = 3 * MAX_SEG;      // vertex queues + chunk queues + far queues
constexpr unsigned FAR_BIT = 0x80000000u;    // in the push buffer: vertex goes to the far queue

// view of queue segment s (segment 0's control block holds the global words:
// pending, abort, error, negcycle, stats)
__device__ __forceinline__ Queue seg_queue(const SolveArgs& a, unsigned s) {
    Queue q = a.q;
    q.slots = a.q.slots + (unsigned long long)s * a.q.N;
    q.ctrl = a.q.ctrl + s;
    return q;
}

__device__ __forceinline__ long long pack_key(long long d, unsigned parent, unsigned shift) {
    return (long long)(((unsigned long long)d << shift) | ((unsigned long long)parent << 1) | 1ull);
}

// ---------------------------------------------------------------------------
// the persistent solver
// ---------------------------------------------------------------------------
// edges of one batch that the edge -> item map covers (bytes per wave);
// MAP = false leaves the map out (the batched solver: its batches are short
// and it keeps the smaller LDS footprint)
template <int B, bool MAP>
constexpr int own_cap() { return MAP ? (B <= 128 ? 8192 : 4096) : 0; }

template <int B, bool MAP = true>
struct WaveLds {
    unsigned item[B];
    int u[B];          // key position of the item's vertex
    unsigned pu[B];    // its original id (CSR row, parent field of candidates)
    long long du[B];
    long long eb[B];
    int pre[B + 1];
    unsigned out[OUTCAP];  // improved vertices to publish
    unsigned hv[OUTCAP];   // the ones with long rows, for the chunk lane
    int fanpre[65];
    alignas(4) unsigned char own[MAP ? own_cap<B, MAP>() : 4];  // batch edge t -> its item
};

// Fill L.own[0, total) with the item each of the batch's first `total`
// edges belongs to: mark every non-empty item's first edge, then carry the
// last mark forward (the marks grow with the position, so it is a running
// maximum), 4 bytes per lane and a DPP wave max-scan per 256 edges. A lookup
// is then one LDS byte read instead of a binary search over the item prefix
// (six dependent reads).
template <class LDS>
__device__ void build_edge_map(LDS& L, unsigned e, int total) {
    const int lane = bq::lane_id();
    unsigned* own32 = reinterpret_cast<unsigned*>(L.own);
    const int words = (total + 3) >> 2;
    for (int i = lane; i < words; i += 64) own32[i] = 0u;
    __builtin_amdgcn_wave_barrier();
    for (unsigned c0 = 0; c0 < e; c0 += 64) {
        const unsigned i = c0 + lane;
        if (i < e && L.pre[i + 1] > L.pre[i] && L.pre[i] < total)
            L.own[L.pre[i]] = (unsigned char)i;
    }
    __builtin_amdgcn_wave_barrier();
    unsigned carry = 0;
    for (int w0 = 0; w0 < words; w0 += 64) {
        const int wi = w0 + lane;
        const unsigned v = wi < words ? own32[wi] : 0u;
        unsigned b0 = v & 255u, b1 = (v >> 8) & 255u, b2 = (v >> 16) & 255u, b3 = v >> 24;
        b1 = b1 > b0 ? b1 : b0;
        b2 = b2 > b1 ? b2 : b1;
        b3 = b3 > b2 ? b3 : b2;
        const unsigned incl = bq::wave_incl_max(b3);
        unsigned prev = bq::wave_shr1(incl);  // lane 0 reads 0
        prev = prev > carry ? prev : carry;
        b0 = b0 > prev ? b0 : prev;
        b1 = b1 > prev ? b1 : prev;
        b2 = b2 > prev ? b2 : prev;
        b3 = b3 > prev ? b3 : prev;
        if (wi < words) own32[wi] = b0 | (b1 << 8) | (b2 << 16) | (b3 << 24);
        const unsigned last = (unsigned)bq::lane63((int)incl);
        carry = last > carry ? last : carry;
    }
    __builtin_amdgcn_wave_barrier();
}

// Publish `cnt` items from the wave's LDS buffer `buf` into queue `seg`
// (Alg. 1 ENQUEUE for all of them at once). The wave's debt (retired items
// not yet subtracted from pending, wave-uniform) pays for the items first;
// pending is raised by the rest before any item becomes visible. Returns
// false on abort.
__device__ bool flush_out(const SolveArgs& a, const Queue& seg, const unsigned* buf, int cnt,
                          long long& debt, unsigned long long& spins) {
    const Queue& q = a.q;
    const int lane = bq::lane_id();
    if (cnt == 0) return true;
    const long long need = (long long)cnt - debt;
    unsigned long long base = 0;
    if (lane == 0) {
        // pending, ENSURE on count and the tail positions as three atomics in
        // flight together. Ordering of the pending raise before the items:
        // the slot stores below are issued only after the wave has the tail
        // atomic's return value (bcast64 waits for it), and gfx9-class
        // hardware (gfx950 included) retires a wave's vector memory
        // operations, no-return atomics among them, in issue order, so by
        // then the pending add has been performed at the device coherence
        // point. A consumer can only retire these items (and subtract them
        // from pending) after reading their slots, so pending never
        // counts them out before it counted them in.
        // In the solver the broker reservation cannot fail:
        // a vertex holds at most one queue item (its q bit) and chunk items
        // are bounded, and each segment holds twice that, so count + cnt <= N
        // always; an overflow would be a bug and stops the solve.
        if (need > 0) bq::add_rlx(&q.ctrl->pending.v, (unsigned long long)need);
        const long long old = bq::add_rlx((BQ_GLOBAL long long*)(&seg.ctrl->count.v),
                                          (long long)cnt);
        base = bq::add_rlx(&seg.ctrl->tail.v, (unsigned long long)cnt);
        if (old + cnt > (long long)seg.N) bq::raise_error(q, bq::ERR_FULL);
    }
    debt = need > 0 ? 0 : -need;
    base = bq::bcast64(base);
    if (bq::aborted(q)) return false;
    for (int c0 = 0; c0 < cnt; c0 += 64) {
        const int i = c0 + lane;
        if (!bq::put_slots(seg, i < cnt, base + (unsigned long long)i, i < cnt ? buf[i] : 0u,
                           a.limit, spins))
            return false;
    }
    return true;
}

// Publish cnt (<= OUTCAP) items with one reservation, as flush_out does for
// 64; the slot words of up to four 64-item slices are read together, so a
// long fan-out costs about one round trip per 256 items instead of three per
// 64. A slice with a slot not yet released takes the waiting path.
__device__ bool flush_many(const SolveArgs& a, const Queue& seg, const unsigned* buf, int cnt,
                           long long& debt, unsigned long long& spins) {
    const Queue& q = a.q;
    const int lane = bq::lane_id();
    if (cnt == 0) return true;
    const long long need = (long long)cnt - debt;
    unsigned long long base = 0;
    if (lane == 0) {
        // the same order of pending, count and tail as in flush_out
        if (need > 0) bq::add_rlx(&q.ctrl->pending.v, (unsigned long long)need);
        const long long old = bq::add_rlx((BQ_GLOBAL long long*)(&seg.ctrl->count.v),
                                          (long long)cnt);
        base = bq::add_rlx(&seg.ctrl->tail.v, (unsigned long long)cnt);
        if (old + cnt > (long long)seg.N) bq::raise_error(q, bq::ERR_FULL);
    }
    debt = need > 0 ? 0 : -need;
    base = bq::bcast64(base);
    if (bq::aborted(q)) return false;
    for (int c0 = 0; c0 < cnt; c0 += 256) {
        unsigned long long w[4];
        for (int r = 0; r < 4; ++r) {
            const int i = c0 + 64 * r + lane;
            w[r] = i < cnt ? bq::ld_rlx(&seg.slots[(base + (unsigned long long)i) & (seg.N - 1ull)])
                           : 0ull;
        }
        for (int r = 0; r < 4; ++r) {
            if (c0 + 64 * r >= cnt) break;
            const int i = c0 + 64 * r + lane;
            const bool act = i < cnt;
            const unsigned long long pos = base + (unsigned long long)i;
            const uint32_t rr = bq::round_of(seg, pos);
            const bool ready = !act || (uint32_t)(w[r] >> 32) == 2u * rr;
            if (__all(ready)) {
                if (act)
                    bq::st_rlx(&seg.slots[pos & (seg.N - 1ull)],
                               bq::slot_word(2u * rr + 1u, buf[i]));
            } else if (!bq::put_slots(seg, act, pos, act ? buf[i] : 0u, a.limit, spins)) {
                return false;
            }
        }
    }
    return true;
}

// Publish the wave's improved vertices (L.out[0, cnt)): entries marked
// FAR_BIT go to the far queue `fq`; with `route`, those with rows longer than
// one chunk go to the chunk lane `cq`; the rest to the vertex queue `hq`.
template <class LDS>
__device__ bool flush_vertices(const SolveArgs& a, const Queue& hq, const Queue& cq,
                               const Queue& fq, LDS& L, int cnt, bool route, long long& debt,
                               unsigned long long& spins) {
    if ((!route && !a.bucket_width) || cnt == 0)
        return flush_out(a, hq, L.out, cnt, debt, spins);
    const int lane = bq::lane_id();
    const long long C = 1ll << a.chunk_log;
    int nl = 0, nh = 0, nf = 0;
    for (int c0 = 0; c0 < cnt; c0 += 64) {
        const int i = c0 + lane;
        const bool live = i < cnt;
        const unsigned x = live ? L.out[i] : 0u;
        const unsigned v = x & ~FAR_BIT;
        const bool far = live && (x & FAR_BIT) != 0u;
        bool hub = false;
        if (route && live && !far) {
            const unsigned ov = orig_of(a, v);
            hub = a.off[ov + 1] - a.off[ov] > C;
        }
        const unsigned long long hm = bq::ballot(hub);
        const unsigned long long fm = bq::ballot(far);
        const unsigned long long lm = bq::ballot(live && !hub && !far);
        // compact in place: a light item moves to an index <= its own, and
        // every lane has read its item before any lane writes; hubs fill
        // L.hv from the front, far items from the back (nh + nf <= cnt)
        if (live && !hub && !far) L.out[nl + bq::rank_in(lm)] = v;
        if (hub) L.hv[nh + bq::rank_in(hm)] = v;
        if (far) L.hv[OUTCAP - 1 - (nf + bq::rank_in(fm))] = v;
        nl += __popcll(lm);
        nh += __popcll(hm);
        nf += __popcll(fm);
    }
    __builtin_amdgcn_wave_barrier();
    if (!flush_out(a, hq, L.out, nl, debt, spins)) return false;
    if (!flush_out(a, cq, L.hv, nh, debt, spins)) return false;
    return flush_out(a, fq, L.hv + (OUTCAP - nf), nf, debt, spins);
}

// Give the wave's debt back to pending (before it waits for work).
__device__ __forceinline__ void pay_debt(const SolveArgs& a, long long& debt) {
    if (debt != 0 && bq::lane_id() == 0)
        bq::add_rlx(&a.q.ctrl->pending.v, (unsigned long long)(-debt));
    debt = 0;
}

// largest idx in [0, e) with pre[idx] <= t (pre[0] = 0, pre non-decreasing)
__device__ __forceinline__ int find_item(const int* pre, int e, int t) {
    int lo = 0, hi = e;  // invariant: pre[lo] <= t < pre[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (pre[mid] <= t)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

// key position of the parent named in x's key (x a key position); the none
// sentinel for unreached and minus-infinity
__device__ __forceinline__ unsigned parent_of(const SolveArgs& a, int x) {
    const long long k = bq::ld_rlx(&a.key[x]);
    const unsigned long long mask = (1ull << (a.shift - 1u)) - 1ull;
    if (is_neg_key(k)) return (unsigned)mask;
    const unsigned p = (unsigned)(((unsigned long long)k >> 1) & mask);
    return p == (unsigned)mask ? p : pos_of(a, p);
}

// minimum weight over edges p -> y, p and y key positions (whole wave scans
// p's row); LLONG_MAX if none
__device__ long long min_edge(const SolveArgs& a, unsigned p, unsigned y) {
    const unsigned pr = orig_of(a, p);
    const long long s = a.off[pr], e = a.off[pr + 1];
    long long best = LLONG_MAX;
    for (long long i = s + bq::lane_id(); i < e; i += 64)
        if ((unsigned)target_of(a, i) == y && weight_of(a, i) < best) best = weight_of(a, i);
    for (int off = 32; off > 0; off >>= 1) {
        const long long o = __shfl_xor(best, off, 64);
        best = o < best ? o : best;
    }
    return (long long)bq::bcast64((unsigned long long)best);
}

// Brent's cycle search on the parent pointers from x0; on a cycle, sum the
// lightest edge of every parent step around it. Returns a vertex of a cycle
// of negative weight, or -1. Wave-uniform.
__device__ int walk_finds_negative_cycle(const SolveArgs& a, int x0, unsigned budget) {
    const unsigned sent = (1u << (a.shift - 1u)) - 1u;
    unsigned power = 1, lam = 1, steps = 0;
    unsigned tort = (unsigned)x0;
    unsigned hare = bq::bcast32(parent_of(a, x0));
    while (tort != hare) {
        if (hare == sent) return -1;
        if (power == lam) {
            tort = hare;
            power <<= 1;
            lam = 0;
        }
        hare = bq::bcast32(parent_of(a, (int)hare));
        ++lam;
        if (++steps > budget) return -1;
        if ((steps & 255u) == 0u && bq::aborted(a.q)) return -1;
    }
    if (hare == sent) return -1;
    // verify: follow lam parent steps from hare, they must close the walk
    long long sum = 0;
    unsigned y = hare;
    for (unsigned i = 0; i < lam; ++i) {
        const unsigned p = bq::bcast32(parent_of(a, (int)y));
        if (p == sent) return -1;
        const long long wmin = min_edge(a, p, y);
        if (wmin == LLONG_MAX) return -1;
        sum += wmin;
        y = p;
    }
    return (y == hare && sum < 0) ? (int)hare : -1;
}

// Per-workgroup parking of idle waves: one wave of the workgroup (the
// poller) watches the global queue state with growing sleeps; the other idle
// waves sleep on workgroup-local flags. This keeps the number of waves
// hammering the hot count / pending lines at one per workgroup.
struct WgShared {
    int poller;     // wave index of the current poller, -1 if none
    unsigned wake;  // bumped by the poller when the count turned positive
    int done;       // pending reached 0: every wave of the workgroup leaves
};

__device__ __forceinline__ int wg_ld(const int* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ unsigned wg_ld(const unsigned* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void wg_st(int* p, int v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Wait for work. Returns 0 when the queue may hold items, 1 when all work is
// done (pending = 0), -1 on abort / watchdog. Wave-uniform.
__device__ int idle_wait(const SolveArgs& a, WgShared& S, int wid, unsigned long long& seen_head,
                         bq::Watch& idle, unsigned long long t_start,
                         unsigned long long& polls) {
    const Queue& q = a.q;
    const int lane = bq::lane_id();
    while (true) {
        if (bq::aborted(q)) return -1;
        if (wg_ld(&S.done)) return 1;
        int got = 0;
        if (lane == 0) {
            int expect = -1;
            got = __hip_atomic_compare_exchange_strong(&S.poller, &expect, wid, __ATOMIC_RELAXED,
                                                       __ATOMIC_RELAXED,
                                                       __HIP_MEMORY_SCOPE_WORKGROUP)
                      ? 1
                      : 0;
        }
        if (bq::bcast32((unsigned)got)) {
            int level = 0;
            while (true) {
                ++polls;
                // lane s < nseg watches segment s; progress = sum of heads
                unsigned long long pend = 0, hd = 0, busy = 0;
                long long cnt = 0;
                if ((unsigned)lane < a.nq) {
                    const bq::Ctrl* c = q.ctrl + lane;
                    cnt = bq::ld_rlx((BQ_GLOBAL const long long*)(&c->count.v));
                    hd = bq::ld_rlx(&c->head.v);
                }
                if (lane == 0) pend = bq::ld_rlx(&q.ctrl->pending.v);
                if (lane == 1 && a.bucket_width) busy = bq::ld_rlx(&q.ctrl->busy.v);
                pend = bq::bcast64(pend);
                busy = (unsigned long long)__shfl((long long)busy, 1, 64);
                // with buckets, far items are work only once no near batch is
                // in flight (the order the far queues are meant to keep)
                const bool far_lane = (unsigned)lane >= 2u * a.nseg;
                const unsigned long long gate =
                    FAR_GATE_PER_WAVE * gridDim.x * (unsigned long long)(blockDim.x >> 6);
                const bool items = __any(cnt > 0 && (!far_lane || busy <= gate));
                for (int off = 32; off > 0; off >>= 1) hd += __shfl_xor(hd, off, 64);
                if (pend == 0ull) {
                    if (lane == 0) {
                        wg_st(&S.done, 1);
                        wg_st(&S.poller, -1);
                    }
                    return 1;
                }
                if (items) {
                    if (lane == 0) {
                        __hip_atomic_fetch_add(&S.wake, 1u, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_WORKGROUP);
                        wg_st(&S.poller, -1);
                    }
                    return 0;
                }
                if (hd != seen_head) {
                    seen_head = hd;
                    idle.arm(a.limit);
                }
                const bool late = idle.expired() || bq::now_ticks() - t_start > a.deadline;
                if (late || bq::aborted(q)) {
                    if (lane == 0) {
                        if (late) bq::raise_error(q, bq::ERR_TIMEOUT);
                        wg_st(&S.poller, -1);
                    }
                    return -1;
                }
                // one poller per workgroup; keep the pollers together at
                // about one poll every 0.2 us on the hot lines
                bq::idle_backoff(level, 8u * gridDim.x);
                if (level < 20) ++level;
            }
        } else {
            const unsigned w0 = wg_ld(&S.wake);
            for (unsigned it = 1;; ++it) {
                __builtin_amdgcn_s_sleep(16);
                if (wg_ld(&S.done)) return 1;
                if (wg_ld(&S.wake) != w0) return 0;
                if (wg_ld(&S.poller) == -1) break;
                if ((it & 63u) == 0u && bq::aborted(q)) return -1;
            }
        }
    }
}

// Work counters of one wave.
struct WaveStats {
    unsigned long long deq, relax, push, fan, batch, walk, impr, spins, idle, poll;
};

// Add a wave's counters to a stats block (lane 0; improvements are per lane).
__device__ inline void flush_stats(bq::Word* stats, WaveStats& st) {
    const int lane = bq::lane_id();
    for (int off = 32; off > 0; off >>= 1) st.impr += __shfl_xor(st.impr, off, 64);
    if (lane == 0) {
        const unsigned long long v[bq::ST_N] = {st.deq,  st.relax, st.push, st.fan,  st.batch,
                                                st.walk, st.spins, st.impr, st.idle, st.poll};
        for (int i = 0; i < bq::ST_N; ++i)
            if (v[i]) bq::add_rlx(&stats[i].v, v[i]);
    }
    st = WaveStats{};
}

// The persistent solver loop of one wave on one query: dequeue a batch,
// stage it, scan its edges, publish improved vertices; until the query's
// pending work is 0 (returns 1) or it is stopped (returns -1). The whole
// workgroup works on the same query; S must be fresh for it. UU edges per
// lane per scan step (U unless the caller picks another).
template <int B, bool MAP, int UU = U>
__device__ int solve_instance(const SolveArgs& a, WaveLds<B, MAP>& L, WgShared& S, int wid,
                              WaveStats& st) {
    const Queue& q = a.q;
    const int lane = bq::lane_id();
    const unsigned shift = a.shift;
    const unsigned clog = a.chunk_log;
    const long long C = 1ll << clog;
    const unsigned n = (unsigned)a.n;

    // weight range -> packing precondition and the negative-cycle bound
    long long wmin = INT_MAX, wmax = INT_MIN;
    {
        const int parts = (int)bq::ld_rlx(&q.ctrl->aux[0].v);
        int lo = INT_MAX, hi = INT_MIN;
        for (int i = lane; i < parts; i += 64) {
            const int x = a.wrange[2 * i], y = a.wrange[2 * i + 1];
            lo = x < lo ? x : lo;
            hi = y > hi ? y : hi;
        }
        for (int off = 32; off > 0; off >>= 1) {
            const int x = __shfl_xor(lo, off, 64), y = __shfl_xor(hi, off, 64);
            lo = x < lo ? x : lo;
            hi = y > hi ? y : hi;
        }
        wmin = lo;
        wmax = hi;
    }
    // segments: home by workgroup (the XCD it runs on); lane s holds the
    // dequeue position where segment s started this solve
    const unsigned home = blockIdx.x % a.nseg;
    const Queue hq = seg_queue(a, home);
    const Queue cq = seg_queue(a, a.nseg + home);  // the chunk lane of this home
    const Queue fq = seg_queue(a, 2u * a.nseg + home);  // its far queue (buckets only)
    const unsigned long long head0_lane =
        (unsigned)lane < a.nq ? bq::ld_rlx(&(q.ctrl + lane)->aux[2].v) : 0ull;
    long long maxabs = 0;
    if (a.m > 0) {
        maxabs = wmax > -wmin ? wmax : -wmin;
        if (maxabs < 0) maxabs = -maxabs;
    }
    // every label of a simple path satisfies |d| <= (n-1) * max|w|; a
    // candidate is at most one more edge away from a checked label
    const double lim = (double)(1ull << (62u - shift));
    if ((double)a.n * (double)maxabs >= lim) {
        if (threadIdx.x == 0) bq::raise_error(q, bq::ERR_RANGE);
        return -1;
    }
    const long long lbound = (long long)(a.n - 1) * (wmin < 0 ? wmin : 0ll);
    // Near / far buckets (bucket_width k > 0): a pushed vertex whose new
    // label is below the threshold T goes to its home's vertex queue, the
    // others to the far queue. Waves take far work only when no vertex or
    // chunk queue has items and few near items are in flight (the `busy`
    // word); the smallest label of a far batch then moves T up to that
    // label + k * max(1, max |w|) / 16 (at least 1). Processing roughly in
    // label order cuts the relabels of large-diameter graphs; the order of
    // work never changes the result.
    long long bdelta = a.bucket_width * (maxabs > 1 ? maxabs : 1ll) / 16;
    if (bdelta < 1) bdelta = 1;
    const unsigned long long far_gate =
        FAR_GATE_PER_WAVE * gridDim.x * (unsigned long long)(blockDim.x >> 6);
    // Row-chunk items a wave takes per batch: about eight scan steps' worth
    // of edges (4096 at UU = 8; 32 chunks of 128, 4 of 1024), at most B. A
    // hub's chunks then spread over more waves instead of a few taking 64
    // each (8192 edges at C = 128): the expansion of the source's and the
    // first hubs' rows, a third of an RMAT-20 solve, ran on a handful of
    // waves (RMAT-20 1.79 -> 1.71 ms, k 2.68 -> 2.47, at 256 workgroups).
    unsigned chunk_take = (8u * 64u * UU) >> clog;
    if (chunk_take < 1u) chunk_take = 1u;
    if (chunk_take > (unsigned)B) chunk_take = (unsigned)B;
    // Parent walks (the negative-cycle search) start once the dequeued work
    // passes suspect_after and then run every walk_stride items. In label
    // order (buckets) a cycle-free solve dequeues about 4 n items, so the
    // search starts at 2 n there, with walks 16 times rarer: road2048 with
    // the planted cycle is flagged in 28 ms instead of 54, and a cycle-free
    // road2048 solve is unchanged (38.5-38.7 ms).
    const bool ordered = a.bucket_width != 0;
    const unsigned long long suspect_after = (ordered ? 2ull : 4ull) * (unsigned long long)a.n +
                                             4ull * (unsigned long long)(a.m >> clog) + 4096ull;
    const unsigned long long walk_stride =
        (unsigned long long)(a.n / 64 > 256 ? a.n / 64 : 256) * (ordered ? 16ull : 1ull);

    const unsigned long long t_start = bq::ld_rlx(&q.ctrl->aux[4].v);

    int result = -1;
    bool had_work = true;  // the first attempt goes straight to the count
    // an idle wave gives up only if the whole queue stops moving (head
    // unchanged for `limit`) while work is still pending
    bq::Watch idle;
    idle.arm(a.limit);
    unsigned long long seen_head = 0;
    long long debt = 0;  // retired items not yet taken off pending (wave-uniform)
    bool flagged = false;  // marking mode: this wave already raised negcycle
    bool long_rows = false;  // this wave has met a row longer than one chunk

    while (true) {
        if (bq::aborted(q)) break;
        if (bq::now_ticks() - t_start > a.deadline) {
            if (lane == 0) bq::raise_error(q, bq::ERR_TIMEOUT);
            break;
        }
        // ---- DEQUEUE up to B items with one reservation -----------------
        // the home chunk lane first, then the home vertex queue; if both are
        // empty, the fullest other queue
        unsigned e = 0;
        unsigned sidx = a.nseg + home;
        if (lane == 0) e = bq::ensure_dequeue(cq, chunk_take, false, a.bwd != 0);
        e = bq::bcast32(e);
        if (e == 0) {
            sidx = home;
            if (lane == 0) e = bq::ensure_dequeue(hq, (unsigned)B, had_work, a.bwd != 0);
            e = bq::bcast32(e);
        }
        if (e == 0) {
            long long c = 0;
            if ((unsigned)lane < 2u * a.nseg && (unsigned)lane != home &&
                (unsigned)lane != a.nseg + home)
                c = bq::ld_rlx((BQ_GLOBAL const long long*)(&(q.ctrl + lane)->count.v));
            // wave arg-max of (count, lane)
            long long best = c > 0 ? c : 0;
            int who = lane;
            for (int off = 32; off > 0; off >>= 1) {
                const long long ob = __shfl_xor(best, off, 64);
                const int ow = __shfl_xor(who, off, 64);
                if (ob > best || (ob == best && ow < who)) {
                    best = ob;
                    who = ow;
                }
            }
            if (best > 0) {
                sidx = bq::bcast32((unsigned)who);
                const unsigned want = sidx >= a.nseg ? chunk_take : (unsigned)B;
                if (lane == 0)
                    e = bq::ensure_dequeue(seg_queue(a, sidx), want, true, a.bwd != 0);
                e = bq::bcast32(e);
            }
        }
        bool far_ok = false;
        if (e == 0 && a.bucket_width) {
            unsigned long long busy = 0;
            if (lane == 0) busy = bq::ld_rlx(&q.ctrl->busy.v);
            far_ok = bq::bcast64(busy) <= far_gate;
        }
        if (e == 0 && far_ok) {
            // no near work queued or in flight: the home far queue, then the
            // fullest other one
            sidx = 2u * a.nseg + home;
            if (lane == 0) e = bq::ensure_dequeue(fq, (unsigned)B, false, a.bwd != 0);
            e = bq::bcast32(e);
            if (e == 0) {
                long long c = 0;
                if ((unsigned)lane >= 2u * a.nseg && (unsigned)lane < a.nq &&
                    (unsigned)lane != 2u * a.nseg + home)
                    c = bq::ld_rlx((BQ_GLOBAL const long long*)(&(q.ctrl + lane)->count.v));
                long long best = c > 0 ? c : 0;
                int who = lane;
                for (int off = 32; off > 0; off >>= 1) {
                    const long long ob = __shfl_xor(best, off, 64);
                    const int ow = __shfl_xor(who, off, 64);
                    if (ob > best || (ob == best && ow < who)) {
                        best = ob;
                        who = ow;
                    }
                }
                if (best > 0) {
                    sidx = bq::bcast32((unsigned)who);
                    if (lane == 0)
                        e = bq::ensure_dequeue(seg_queue(a, sidx), (unsigned)B, true,
                                               a.bwd != 0);
                    e = bq::bcast32(e);
                }
            }
        }
        const Queue dq = seg_queue(a, sidx);
        unsigned long long base = 0;
        const bool near_batch = a.bucket_width && e && sidx < 2u * a.nseg;
        if (e && lane == 0) {
            if (near_batch) bq::add_rlx(&q.ctrl->busy.v, (unsigned long long)e);
            base = bq::add_rlx(&dq.ctrl->head.v, (unsigned long long)e);
        }
        had_work = e > 0 && sidx == home;
        if (e == 0) {
            ++st.idle;
            pay_debt(a, debt);
            const int r = idle_wait(a, S, wid, seen_head, idle, t_start, st.poll);
            if (r != 0) {
                result = r;
                break;
            }
            had_work = true;  // the poller saw a positive count
            continue;
        }
        idle.arm(a.limit);
        base = bq::bcast64(base);
        ++st.batch;
        st.deq += e;
        bool ok = true;
        bool any_chunk = false;
        for (unsigned c0 = 0; c0 < e; c0 += 64) {
            const unsigned i = c0 + lane;
            unsigned v = 0;
            if (!bq::read_slots(dq, i < e, base + i, v, a.limit, st.spins)) {
                ok = false;
                break;
            }
            if (i < e) L.item[i] = v;
            any_chunk |= __any(i < e && v >= n);
        }
        if (!ok) break;
        // chunk items name their row through chunk_owner, written before
        // the items were published (see the fan-out below)
        long_rows |= any_chunk;
        if (a.trace && sidx == 0) {  // timeline of the vertex queue (one segment)
            const unsigned long long w0 = base - head0_lane, w1 = w0 + e;
            if ((w0 >> a.trace_shift) != (w1 >> a.trace_shift) && lane == 0) {
                const unsigned long long idx = w1 >> a.trace_shift;
                if (idx < a.trace_cap) {
                    unsigned long long* t = a.trace + 4ull * idx;
                    t[0] = bq::now_ticks() - t_start;
                    t[1] = w1;
                    t[2] = bq::ld_rlx(&q.ctrl->tail.v) - bq::ld_rlx(&q.ctrl->head.v);
                    t[3] = bq::ld_rlx(&q.ctrl->pending.v);
                }
            }
        }

        // ---- stage the batch: label, edge range, row chunks --------------
        int carry = 0;
        int fan_total = 0;
        for (unsigned c0 = 0; c0 < e; c0 += 64) {
            const unsigned i = c0 + lane;
            int cnt = 0, fan = 0;
            if (i < e) {
                const unsigned it = L.item[i];
                int u;
                unsigned ur;
                long long d, s, t;
                if (it < n) {
                    u = (int)it;
                    const long long old = __hip_atomic_fetch_and(
                        &a.key[u], ~1ll, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    d = old >> shift;
                    ur = orig_of(a, (unsigned)u);
                    s = a.off[ur];
                    t = a.off[ur + 1];
                    if (t - s > C) {
                        const long long js = s >> clog, je = (t - 1) >> clog;
                        t = (js + 1) << clog;
                        fan = (int)(je - js);
                    }
                } else {
                    const long long j = (long long)(it - n);
                    u = (int)bq::ld_rlx(&a.chunk_owner[j]);
                    d = bq::ld_rlx(&a.key[u]) >> shift;
                    ur = orig_of(a, (unsigned)u);
                    const long long r0 = a.off[ur], r1 = a.off[ur + 1];
                    s = j << clog;
                    t = (j + 1) << clog;
                    s = s > r0 ? s : r0;
                    t = t < r1 ? t : r1;
                }
                L.u[i] = u;
                L.pu[i] = ur;
                L.du[i] = d;
                L.eb[i] = s;
                cnt = (int)(t - s);
            }
            const int incl = bq::wave_incl_scan(cnt);
            if (i < e) L.pre[i + 1] = carry + incl;
            carry += bq::lane63(incl);
            // fan-out of this 64-item slice: lanes with hubs publish the later
            // chunks of their rows
            const int fincl = bq::wave_incl_scan(fan);
            const int ftot = bq::lane63(fincl);
            if (ftot > 0) {
                L.fanpre[lane + 1] = fincl;
                if (lane == 0) L.fanpre[0] = 0;
                __builtin_amdgcn_wave_barrier();
                int nbuf = 0;  // chunk items in L.out not yet published
                for (int t0 = 0; t0 < ftot; t0 += 64) {
                    const int k = t0 + lane;
                    // chunk items go through the LDS buffer, 64 per pass
                    // (with fan_bulk, up to OUTCAP before they are published)
                    if (k < ftot) {
                        int lo = 0, hi = 64;
                        while (hi - lo > 1) {
                            const int mid = (lo + hi) >> 1;
                            if (L.fanpre[mid] <= k) lo = mid; else hi = mid;
                        }
                        const unsigned owner_item = c0 + (unsigned)lo;
                        const int ou = L.u[owner_item];
                        const long long js = L.eb[owner_item] >> clog;
                        const long long j = js + 1 + (k - L.fanpre[lo]);
                        // an agent-scope store, like the slot words: it is
                        // complete at the device coherence point before the
                        // chunk items' slot stores are issued (those wait for
                        // the tail ticket, and one wave's vector memory
                        // operations retire in issue order), and the taker
                        // reads it with an agent-scope load that depends on
                        // the slot's value. (An L2 write-back / invalidate
                        // fence pair instead cost 5-8 %.)
                        bq::st_rlx(&a.chunk_owner[j], (unsigned)ou);
                        L.out[nbuf + lane] = (unsigned)(n + (unsigned)j);
                    }
                    nbuf += (ftot - t0) < 64 ? (ftot - t0) : 64;
                    if (a.fan_bulk && nbuf <= OUTCAP - 64 && t0 + 64 < ftot) continue;
                    __builtin_amdgcn_wave_barrier();
                    if (!(a.fan_bulk ? flush_many(a, cq, L.out, nbuf, debt, st.spins)
                                     : flush_out(a, cq, L.out, nbuf, debt, st.spins))) {
                        ok = false;
                        break;
                    }
                    nbuf = 0;
                    __builtin_amdgcn_wave_barrier();
                }
                fan_total += ftot;
                long_rows = true;
                if (!ok) break;
            }
        }
        if (!ok) break;
        st.fan += (unsigned long long)fan_total;
        if (lane == 0) L.pre[0] = 0;
        __builtin_amdgcn_wave_barrier();
        if (sidx >= 2u * a.nseg) {
            // a far batch: T moves up to its smallest label + the bucket width
            long long lo = LLONG_MAX;
            for (unsigned i = lane; i < e; i += 64) lo = L.du[i] < lo ? L.du[i] : lo;
            for (int off = 32; off > 0; off >>= 1) {
                const long long o = __shfl_xor(lo, off, 64);
                lo = o < lo ? o : lo;
            }
            if (lane == 0 && lo < LLONG_MAX - bdelta)
                __hip_atomic_fetch_max((BQ_GLOBAL long long*)&q.ctrl->aux[1].v, lo + bdelta,
                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        // the threshold this batch's pushes are split at
        const long long tsplit =
            a.bucket_width ? (long long)bq::bcast64(bq::ld_rlx(&q.ctrl->aux[1].v)) : LLONG_MAX;

        // ---- scan the concatenated edge range ---------------------------
        // Three-stage software pipeline over groups of 64*UU edges: in each
        // step the wave issues the atomics of group g, the key loads of group
        // g+1 and the target/weight loads of group g+2, and waits once.
        // An atomicMin is issued only when the candidate is below the key
        // loaded one step earlier: keys only decrease, so a candidate that is
        // not below an earlier value of the key cannot change it, and the
        // atomic would be a no-op. Most relaxations are such no-ops, and on
        // high in-degree targets the atomics would otherwise serialize.
        const int total = carry;
        st.relax += (unsigned long long)total;
        // edges [0, mapped) find their item in the map, any later ones by a
        // binary search; a batch that fits one step searches (the map would
        // cost more than it saves)
        constexpr int cap = own_cap<B, MAP>();
        const int mapped = (!MAP || total <= 64 * UU) ? 0 : (total < cap ? total : cap);
        if constexpr (MAP) {
            if (mapped > 0) build_edge_map(L, e, mapped);
        }
        int nout = 0;
        int av[UU], aw[UU], aidx[UU];           // group g+2: target, weight, item
        int bv[UU], bw[UU], bidx[UU];           // group g+1
        long long bkey[UU];
        auto fetch = [&](int t0) {
#pragma unroll
            for (int r = 0; r < UU; ++r) {
                const int t = t0 + r * 64 + lane;
                av[r] = -1;
                aw[r] = 0;
                aidx[r] = 0;
                if (t < total) {
                    const int idx = t < mapped ? (int)L.own[t] : find_item(L.pre, (int)e, t);
                    const long long edge = L.eb[idx] + (t - L.pre[idx]);
                    aidx[r] = idx;
                    av[r] = target_of(a, edge);
                    aw[r] = weight_of(a, edge);
                }
            }
        };
        // a batch that fits one step skips the key check: there the extra
        // load would only add a round trip
        const bool check = total > 64 * UU;
        auto advance = [&]() {  // stage A -> stage B, issuing B's key loads
#pragma unroll
            for (int r = 0; r < UU; ++r) {
                bv[r] = av[r];
                bw[r] = aw[r];
                bidx[r] = aidx[r];
                bkey[r] = bv[r] < 0 ? LLONG_MIN
                                    : (check ? bq::ld_rlx(&a.key[bv[r]]) : LLONG_MAX);
            }
        };
        fetch(0);
        advance();
        if (64 * UU < total) fetch(64 * UU);
        for (int t0 = 0; t0 < total && ok; t0 += 64 * UU) {
            long long cand[UU], cd[UU], seen[UU];
            int tv[UU];
            bool valid[UU];
#pragma unroll
            for (int r = 0; r < UU; ++r) {
                tv[r] = bv[r];
                valid[r] = tv[r] >= 0;
                seen[r] = bkey[r];
                cd[r] = L.du[bidx[r]] + (long long)bw[r];
                cand[r] = pack_key(cd[r], L.pu[bidx[r]], shift);
                // marking mode: a candidate below the certain lower bound (or
                // from a minus-infinity source, whose label is far below it)
                // proves that a negative cycle reaches the target
                if (a.neginf && cd[r] < lbound) cand[r] = KEY_NEG;
            }
            if (t0 + 64 * UU < total) advance();
            if (t0 + 128 * UU < total) fetch(t0 + 128 * UU);
            long long old[UU];
#pragma unroll
            for (int r = 0; r < UU; ++r) {
                const bool try_it = valid[r] && cand[r] < seen[r];
                valid[r] = try_it;
                old[r] = try_it ? __hip_atomic_fetch_min(&a.key[tv[r]], cand[r], __ATOMIC_RELAXED,
                                                         __HIP_MEMORY_SCOPE_AGENT)
                                : LLONG_MIN;
            }
            bool neg = false;
#pragma unroll
            for (int r = 0; r < UU; ++r) {
                const bool won = valid[r] && cand[r] < old[r];
                const bool dropped = won && cd[r] < (old[r] >> shift);
                st.impr += dropped;
                neg |= dropped && cd[r] < lbound;
                const bool push = won && (old[r] & 1ll) == 0;
                const unsigned long long pm = bq::ballot(push);
                if (push)
                    L.out[nout + bq::rank_in(pm)] =
                        (unsigned)tv[r] | (cd[r] >= tsplit ? FAR_BIT : 0u);
                nout += __popcll(pm);
            }
            if (__any(neg)) {
                if (!a.neginf) {
                    if (lane == 0) {
                        bq::st_rlx(&q.ctrl->negcycle.v, 1ull);
                        bq::st_rlx(&q.ctrl->abort.v, 1ull);
                    }
                    ok = false;
                    break;
                }
                if (!flagged && lane == 0) bq::st_rlx(&q.ctrl->negcycle.v, 1ull);
                flagged = true;
            }
            if (nout > OUTCAP - 64 * UU) {
                __builtin_amdgcn_wave_barrier();
                if (!flush_vertices(a, hq, cq, fq, L, nout, long_rows, debt, st.spins)) {
                    ok = false;
                    break;
                }
                st.push += (unsigned long long)nout;
                nout = 0;
                __builtin_amdgcn_wave_barrier();
            }
        }
        if (!ok) break;
        __builtin_amdgcn_wave_barrier();
        // retire this batch into the debt, then publish the rest
        debt += (long long)e;
        if (!flush_vertices(a, hq, cq, fq, L, nout, long_rows, debt, st.spins)) break;
        st.push += (unsigned long long)nout;
        // its pushes are queued: the near batch is no longer in flight
        if (near_batch && lane == 0)
            bq::add_rlx(&q.ctrl->busy.v, (unsigned long long)(-(long long)e));

        // ---- negative-cycle search once the work looks unbounded --------
        // work so far, estimated from this segment's dequeue position
        const unsigned long long h0 = bq::bcast64(__shfl(head0_lane, (int)sidx, 64));
        const unsigned long long work = (base + e - h0) * a.nseg;
        const unsigned long long prev = (base - h0) * a.nseg;
        if (work > suspect_after && prev / walk_stride != work / walk_stride) {
            ++st.walk;
            const unsigned budget = (unsigned)(a.n < (1 << 20) ? a.n + 1 : (1 << 20));
            const int hit = walk_finds_negative_cycle(a, L.u[0], budget);
            if (hit >= 0 && !a.neginf) {
                if (lane == 0) {
                    bq::st_rlx(&q.ctrl->negcycle.v, 1ull);
                    bq::st_rlx(&q.ctrl->abort.v, 1ull);
                }
                break;
            }
            if (hit >= 0) {
                // marking mode: the cycle's vertex becomes minus infinity and
                // spreads it through the queue like any lowered label
                long long old = 0;
                if (lane == 0) {
                    old = __hip_atomic_fetch_min(&a.key[hit], KEY_NEG, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT);
                    if (!flagged) bq::st_rlx(&q.ctrl->negcycle.v, 1ull);
                }
                flagged = true;
                old = (long long)bq::bcast64((unsigned long long)old);
                const int cnt = (KEY_NEG < old && (old & 1ll) == 0) ? 1 : 0;
                if (lane == 0) L.out[0] = (unsigned)hit;
                __builtin_amdgcn_wave_barrier();
                if (!flush_out(a, hq, L.out, cnt, debt, st.spins)) break;
                st.push += (unsigned long long)cnt;
            }
        }
    }

    return result;
}

}  // namespace
