// Queue-based Bellman-Ford SSSP on one gfx950 device (Section III.C), driven
// by the Broker Queue of Section III.A.
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
// Termination: `pending` counts items enqueued or being processed; a wave
// leaves when the queue is empty and pending is 0.
//
// Negative cycles (Alg. 3 detects them as changes in round n-1; a queue has
// no rounds): (1) a label below (n-1) * min(0, min w) is impossible without
// one; (2) once the dequeued work exceeds a few times n, some waves walk the
// parent pointers (Brent's cycle finding); a closed walk of real edges whose
// weights sum below zero proves a negative cycle reachable from src.
#include <hip/hip_runtime.h>
#include <limits.h>
#include <stdio.h>
#include <stdlib.h>

#include "host_common.hpp"

using bq::Queue;

namespace {

constexpr long long KEY_INF = 0x7FFFFFFFFFFFFFFELL;  // d = max, parent = all ones, q = 0
constexpr int SOLVE_WG = 256;
constexpr int WAVES_PER_WG = SOLVE_WG / 64;
constexpr int OUTCAP = 1024;  // LDS push buffer per wave
#ifndef SSSP_UNROLL
#define SSSP_UNROLL 8
#endif
constexpr int U = SSSP_UNROLL;  // edges per lane per pipelined step

struct SolveArgs {
    Queue q;
    const long long* off;
    const int* col;
    const int* w;
    long long* key;          // the caller's dist buffer, used as key array
    unsigned* chunk_owner;   // [m >> chunk_log + 1]
    const int* wrange;       // per-block (min w, max w) from k_init
    int n;
    int src;
    long long m;
    unsigned shift;          // S = PB + 1
    unsigned chunk_log;
    unsigned long long limit;     // one wait (ticks of the 100 MHz clock)
    unsigned long long deadline;  // whole solve
    unsigned long long* trace;    // optional timeline: 4 words per sample
    unsigned trace_shift;         // one sample per 2^trace_shift dequeued items
    unsigned trace_cap;           // samples
};

__device__ __forceinline__ long long pack_key(long long d, unsigned parent, unsigned shift) {
    return (long long)(((unsigned long long)d << shift) | ((unsigned long long)parent << 1) | 1ull);
}

// ---------------------------------------------------------------------------
// init: keys, the per-block weight range, and (block 0) the control block
// with the source already enqueued
// ---------------------------------------------------------------------------
constexpr int INIT_WG = 256;
constexpr int INIT_MAX_BLOCKS = 1024;

__global__ __launch_bounds__(INIT_WG) void k_init(Queue q, long long* key, int n, int src,
                                                  unsigned shift, const int* w, long long m,
                                                  int* wrange /* [2 * gridDim.x] */) {
    const long long tid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long stride = (long long)gridDim.x * blockDim.x;
    const long long srckey = pack_key(0, (1u << (shift - 1u)) - 1u, shift);
    for (long long v = tid; v < n; v += stride) key[v] = (v == src) ? srckey : KEY_INF;
    int lo = INT_MAX, hi = INT_MIN;
    for (long long e = tid; e < m; e += stride) {
        const int x = w[e];
        lo = x < lo ? x : lo;
        hi = x > hi ? x : hi;
    }
    for (int off = 32; off > 0; off >>= 1) {
        const int a2 = __shfl_xor(lo, off, 64), b2 = __shfl_xor(hi, off, 64);
        lo = a2 < lo ? a2 : lo;
        hi = b2 > hi ? b2 : hi;
    }
    __shared__ int slo[INIT_WG / 64], shi[INIT_WG / 64];
    if (bq::lane_id() == 0) {
        slo[threadIdx.x >> 6] = lo;
        shi[threadIdx.x >> 6] = hi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < INIT_WG / 64; ++i) {
            lo = slo[i] < lo ? slo[i] : lo;
            hi = shi[i] > hi ? shi[i] : hi;
        }
        wrange[2 * blockIdx.x] = lo;
        wrange[2 * blockIdx.x + 1] = hi;
    }
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    bq::Ctrl* c = q.ctrl;
    c->pending.v = 1ull;
    c->abort.v = 0ull;
    c->error.v = 0ull;
    c->negcycle.v = 0ull;
    c->aux[0].v = (unsigned long long)gridDim.x;  // number of weight-range partials
    c->aux[2].v = c->head.v;                      // dequeue position at start
    c->aux[4].v = bq::now_ticks();                // clock at start
    for (int i = 0; i < bq::ST_N; ++i) c->stats[i].v = 0ull;
    // enqueue src: the queue is quiescent, so slot (tail mod N) is free for
    // this round (ticket 2r) and count is 0
    const unsigned long long pos = c->tail.v;
    const unsigned slot = (unsigned)(pos & (q.N - 1ull));
    const unsigned round = (unsigned)(pos >> q.logN);
    q.slots[slot] = bq::slot_word(2u * round + 1u, (unsigned)src);
    c->tail.v = pos + 1ull;
    c->count.v = 1ull;
}

// CSR checks (flag BQ_F_VALIDATE): aux[3] becomes non-zero on a defect.
__global__ void k_validate(const long long* off, const int* col, int n, long long m,
                           bq::Ctrl* ctrl) {
    const long long tid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long stride = (long long)gridDim.x * blockDim.x;
    bool bad = false;
    if (tid == 0) bad = off[0] != 0 || off[n] != m;
    for (long long v = tid; v < n; v += stride) bad |= off[v + 1] < off[v];
    for (long long e = tid; e < m; e += stride) bad |= (unsigned)col[e] >= (unsigned)n;
    if (__any(bad) && bq::lane_id() == 0) bq::st_rlx(&ctrl->aux[3].v, 1ull);
}

// ---------------------------------------------------------------------------
// the persistent solver
// ---------------------------------------------------------------------------
template <int B>
struct WaveLds {
    unsigned item[B];
    int u[B];
    long long du[B];
    long long eb[B];
    int pre[B + 1];
    unsigned out[OUTCAP];
    int fanpre[65];
};

// Publish `cnt` items from the wave's LDS buffer (Alg. 1 ENQUEUE for all of
// them at once). pending is raised by `cnt + pending_delta` before any item
// becomes visible. `release` orders earlier plain stores (the chunk table)
// before the items. Returns false on abort.
template <class LDS>
__device__ bool flush_out(const SolveArgs& a, LDS& L, int cnt, long long pending_delta,
                          bool release, unsigned long long& spins) {
    const Queue& q = a.q;
    const int lane = bq::lane_id();
    if (cnt == 0) {
        if (pending_delta != 0 && lane == 0)
            bq::add_rlx(&q.ctrl->pending.v, (unsigned long long)pending_delta);
        return true;
    }
    unsigned long long base = 0;
    if (lane == 0) {
        // pending, ENSURE on count and the tail positions as three atomics in
        // flight together. In the solver the broker reservation cannot fail:
        // a vertex holds at most one queue item (its q bit) and chunk items
        // are bounded, and the capacity is twice that, so count + cnt <= N
        // always; an overflow would be a bug and stops the solve.
        bq::add_rlx(&q.ctrl->pending.v, (unsigned long long)((long long)cnt + pending_delta));
        const long long old = bq::add_rlx(reinterpret_cast<long long*>(&q.ctrl->count.v),
                                          (long long)cnt);
        base = bq::add_rlx(&q.ctrl->tail.v, (unsigned long long)cnt);
        if (old + cnt > (long long)q.N) bq::raise_error(q, bq::ERR_FULL);
    }
    base = bq::bcast64(base);
    if (bq::aborted(q)) return false;
    if (release) bq::fence_release();
    for (int c0 = 0; c0 < cnt; c0 += 64) {
        const int i = c0 + lane;
        if (!bq::put_slots(q, i < cnt, base + (unsigned long long)i, i < cnt ? L.out[i] : 0u,
                           a.limit, spins))
            return false;
    }
    return true;
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

__device__ __forceinline__ unsigned parent_of(const SolveArgs& a, int x) {
    const unsigned long long k = (unsigned long long)bq::ld_rlx(&a.key[x]);
    return (unsigned)((k >> 1) & ((1ull << (a.shift - 1u)) - 1ull));
}

// minimum weight over edges p -> y (whole wave scans row p); LLONG_MAX if none
__device__ long long min_edge(const SolveArgs& a, unsigned p, unsigned y) {
    const long long s = a.off[p], e = a.off[p + 1];
    long long best = LLONG_MAX;
    for (long long i = s + bq::lane_id(); i < e; i += 64)
        if ((unsigned)a.col[i] == y && a.w[i] < best) best = a.w[i];
    for (int off = 32; off > 0; off >>= 1) {
        const long long o = __shfl_xor(best, off, 64);
        best = o < best ? o : best;
    }
    return (long long)bq::bcast64((unsigned long long)best);
}

// Brent's cycle search on the parent pointers from x0; on a cycle, sum the
// lightest edge of every parent step around it. Wave-uniform.
__device__ bool walk_finds_negative_cycle(const SolveArgs& a, int x0, unsigned budget) {
    const unsigned sent = (1u << (a.shift - 1u)) - 1u;
    unsigned power = 1, lam = 1, steps = 0;
    unsigned tort = (unsigned)x0;
    unsigned hare = bq::bcast32(parent_of(a, x0));
    while (tort != hare) {
        if (hare == sent) return false;
        if (power == lam) {
            tort = hare;
            power <<= 1;
            lam = 0;
        }
        hare = bq::bcast32(parent_of(a, (int)hare));
        ++lam;
        if (++steps > budget) return false;
        if ((steps & 255u) == 0u && bq::aborted(a.q)) return false;
    }
    if (hare == sent) return false;
    // verify: follow lam parent steps from hare, they must close the walk
    long long sum = 0;
    unsigned y = hare;
    for (unsigned i = 0; i < lam; ++i) {
        const unsigned p = bq::bcast32(parent_of(a, (int)y));
        if (p == sent) return false;
        const long long wmin = min_edge(a, p, y);
        if (wmin == LLONG_MAX) return false;
        sum += wmin;
        y = p;
    }
    return y == hare && sum < 0;
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
                unsigned long long pend = 0, cnt = 0, hd = 0;
                if (lane == 0) {
                    pend = bq::ld_rlx(&q.ctrl->pending.v);
                    cnt = bq::ld_rlx(&q.ctrl->count.v);
                    hd = bq::ld_rlx(&q.ctrl->head.v);
                }
                pend = bq::bcast64(pend);
                cnt = bq::bcast64(cnt);
                hd = bq::bcast64(hd);
                if (pend == 0ull) {
                    if (lane == 0) {
                        wg_st(&S.done, 1);
                        wg_st(&S.poller, -1);
                    }
                    return 1;
                }
                if ((long long)cnt > 0) {
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

template <int B>
__global__ __launch_bounds__(SOLVE_WG) void k_solve(SolveArgs a) {
    __shared__ WaveLds<B> lds[WAVES_PER_WG];
    __shared__ WgShared S;
    WaveLds<B>& L = lds[threadIdx.x >> 6];
    const int wid = (int)(threadIdx.x >> 6);
    if (threadIdx.x == 0) {
        S.poller = -1;
        S.wake = 0u;
        S.done = 0;
    }
    __syncthreads();
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
    const unsigned long long head0 = bq::ld_rlx(&q.ctrl->aux[2].v);
    long long maxabs = 0;
    if (a.m > 0) {
        maxabs = wmax > -wmin ? wmax : -wmin;
        if (maxabs < 0) maxabs = -maxabs;
    }
    // every label of a simple path satisfies |d| <= (n-1) * max|w|; a
    // candidate is at most one more edge away from a checked label
    const double lim = (double)(1ull << (62u - shift));
    if ((double)a.n * (double)maxabs >= lim) {
        if (lane == 0 && blockIdx.x == 0 && threadIdx.x == 0) bq::raise_error(q, bq::ERR_RANGE);
        return;
    }
    const long long lbound = (long long)(a.n - 1) * (wmin < 0 ? wmin : 0ll);
    const unsigned long long suspect_after = 4ull * (unsigned long long)a.n +
                                             4ull * (unsigned long long)(a.m >> clog) + 4096ull;
    const unsigned long long walk_stride =
        (unsigned long long)(a.n / 64 > 256 ? a.n / 64 : 256);

    const unsigned long long t_start = bq::ld_rlx(&q.ctrl->aux[4].v);

    unsigned long long st_deq = 0, st_relax = 0, st_push = 0, st_fan = 0, st_batch = 0,
                       st_walk = 0, st_impr = 0, spins = 0, st_idle = 0, st_poll = 0;
    bool had_work = true;  // the first attempt goes straight to the count
    // an idle wave gives up only if the whole queue stops moving (head
    // unchanged for `limit`) while work is still pending
    bq::Watch idle;
    idle.arm(a.limit);
    unsigned long long seen_head = 0;

    while (true) {
        if (bq::aborted(q)) break;
        if (bq::now_ticks() - t_start > a.deadline) {
            if (lane == 0) bq::raise_error(q, bq::ERR_TIMEOUT);
            break;
        }
        // ---- DEQUEUE up to B items with one reservation -----------------
        unsigned e = 0;
        unsigned long long base = 0;
        if (lane == 0) {
            e = bq::reserve_dequeue(q, (unsigned)B, had_work);
            if (e) base = bq::add_rlx(&q.ctrl->head.v, (unsigned long long)e);
        }
        e = bq::bcast32(e);
        had_work = e > 0;
        if (e == 0) {
            ++st_idle;
            if (idle_wait(a, S, wid, seen_head, idle, t_start, st_poll) != 0) break;
            had_work = true;  // the poller saw a positive count
            continue;
        }
        idle.arm(a.limit);
        base = bq::bcast64(base);
        ++st_batch;
        st_deq += e;
        bool ok = true;
        bool any_chunk = false;
        for (unsigned c0 = 0; c0 < e; c0 += 64) {
            const unsigned i = c0 + lane;
            unsigned v = 0;
            if (!bq::read_slots(q, i < e, base + i, v, a.limit, spins)) {
                ok = false;
                break;
            }
            if (i < e) L.item[i] = v;
            any_chunk |= __any(i < e && v >= n);
        }
        if (!ok) break;
        // chunk items name their row through chunk_owner, written before
        // the items were published (release fence on that side)
        if (any_chunk) bq::fence_acquire();
        if (a.trace) {
            const unsigned long long w0 = base - head0, w1 = w0 + e;
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
                long long d, s, t;
                if (it < n) {
                    u = (int)it;
                    const long long old = __hip_atomic_fetch_and(
                        &a.key[u], ~1ll, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    d = old >> shift;
                    s = a.off[u];
                    t = a.off[u + 1];
                    if (t - s > C) {
                        const long long js = s >> clog, je = (t - 1) >> clog;
                        t = (js + 1) << clog;
                        fan = (int)(je - js);
                    }
                } else {
                    const long long j = (long long)(it - n);
                    u = (int)bq::ld_rlx(&a.chunk_owner[j]);
                    d = bq::ld_rlx(&a.key[u]) >> shift;
                    const long long r0 = a.off[u], r1 = a.off[u + 1];
                    s = j << clog;
                    t = (j + 1) << clog;
                    s = s > r0 ? s : r0;
                    t = t < r1 ? t : r1;
                }
                L.u[i] = u;
                L.du[i] = d;
                L.eb[i] = s;
                cnt = (int)(t - s);
            }
            const int incl = bq::wave_incl_scan(cnt);
            if (i < e) L.pre[i + 1] = carry + incl;
            carry += __shfl(incl, 63, 64);
            // fan-out of this 64-item slice: lanes with hubs publish the later
            // chunks of their rows
            const int fincl = bq::wave_incl_scan(fan);
            const int ftot = __shfl(fincl, 63, 64);
            if (ftot > 0) {
                L.fanpre[lane + 1] = fincl;
                if (lane == 0) L.fanpre[0] = 0;
                __builtin_amdgcn_wave_barrier();
                for (int t0 = 0; t0 < ftot; t0 += 64) {
                    const int k = t0 + lane;
                    // chunk items go through the LDS buffer (at most 64 here)
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
                        a.chunk_owner[j] = (unsigned)ou;
                        L.out[lane] = (unsigned)(n + (unsigned)j);
                    }
                    const int cnt_now = (ftot - t0) < 64 ? (ftot - t0) : 64;
                    __builtin_amdgcn_wave_barrier();
                    if (!flush_out(a, L, cnt_now, 0, true, spins)) {
                        ok = false;
                        break;
                    }
                    __builtin_amdgcn_wave_barrier();
                }
                fan_total += ftot;
                if (!ok) break;
            }
        }
        if (!ok) break;
        st_fan += (unsigned long long)fan_total;
        if (lane == 0) L.pre[0] = 0;
        __builtin_amdgcn_wave_barrier();

        // ---- scan the concatenated edge range ---------------------------
        // Three-stage software pipeline over groups of 64*U edges: in each
        // step the wave issues the atomics of group g, the key loads of group
        // g+1 and the target/weight loads of group g+2, and waits once.
        // An atomicMin is issued only when the candidate is below the key
        // loaded one step earlier: keys only decrease, so a candidate that is
        // not below an earlier value of the key cannot change it, and the
        // atomic would be a no-op. Most relaxations are such no-ops, and on
        // high in-degree targets the atomics would otherwise serialize.
        const int total = carry;
        st_relax += (unsigned long long)total;
        int nout = 0;
        int av[U], aw[U], aidx[U];           // group g+2: target, weight, item
        int bv[U], bw[U], bidx[U];           // group g+1
        long long bkey[U];
        auto fetch = [&](int t0) {
#pragma unroll
            for (int r = 0; r < U; ++r) {
                const int t = t0 + r * 64 + lane;
                av[r] = -1;
                aw[r] = 0;
                aidx[r] = 0;
                if (t < total) {
                    const int idx = find_item(L.pre, (int)e, t);
                    const long long edge = L.eb[idx] + (t - L.pre[idx]);
                    aidx[r] = idx;
                    av[r] = a.col[edge];
                    aw[r] = a.w[edge];
                }
            }
        };
        // a batch that fits one step skips the key check: there the extra
        // load would only add a round trip
        const bool check = total > 64 * U;
        auto advance = [&]() {  // stage A -> stage B, issuing B's key loads
#pragma unroll
            for (int r = 0; r < U; ++r) {
                bv[r] = av[r];
                bw[r] = aw[r];
                bidx[r] = aidx[r];
                bkey[r] = bv[r] < 0 ? LLONG_MIN
                                    : (check ? bq::ld_rlx(&a.key[bv[r]]) : LLONG_MAX);
            }
        };
        fetch(0);
        advance();
        if (64 * U < total) fetch(64 * U);
        for (int t0 = 0; t0 < total && ok; t0 += 64 * U) {
            long long cand[U], cd[U], seen[U];
            int tv[U];
            bool valid[U];
#pragma unroll
            for (int r = 0; r < U; ++r) {
                tv[r] = bv[r];
                valid[r] = tv[r] >= 0;
                seen[r] = bkey[r];
                cd[r] = L.du[bidx[r]] + (long long)bw[r];
                cand[r] = pack_key(cd[r], (unsigned)L.u[bidx[r]], shift);
            }
            if (t0 + 64 * U < total) advance();
            if (t0 + 128 * U < total) fetch(t0 + 128 * U);
            long long old[U];
#pragma unroll
            for (int r = 0; r < U; ++r) {
                const bool try_it = valid[r] && cand[r] < seen[r];
                valid[r] = try_it;
                old[r] = try_it ? __hip_atomic_fetch_min(&a.key[tv[r]], cand[r], __ATOMIC_RELAXED,
                                                         __HIP_MEMORY_SCOPE_AGENT)
                                : LLONG_MIN;
            }
            bool neg = false;
#pragma unroll
            for (int r = 0; r < U; ++r) {
                const bool won = valid[r] && cand[r] < old[r];
                const bool dropped = won && cd[r] < (old[r] >> shift);
                st_impr += dropped;
                neg |= dropped && cd[r] < lbound;
                const bool push = won && (old[r] & 1ll) == 0;
                const unsigned long long pm = bq::ballot(push);
                if (push) L.out[nout + bq::rank_in(pm)] = (unsigned)tv[r];
                nout += __popcll(pm);
            }
            if (__any(neg)) {
                if (lane == 0) {
                    bq::st_rlx(&q.ctrl->negcycle.v, 1ull);
                    bq::st_rlx(&q.ctrl->abort.v, 1ull);
                }
                ok = false;
                break;
            }
            if (nout > OUTCAP - 64 * U) {
                __builtin_amdgcn_wave_barrier();
                if (!flush_out(a, L, nout, 0, false, spins)) {
                    ok = false;
                    break;
                }
                st_push += (unsigned long long)nout;
                nout = 0;
                __builtin_amdgcn_wave_barrier();
            }
        }
        if (!ok) break;
        __builtin_amdgcn_wave_barrier();
        // publish the rest and retire this batch in one pending update
        if (!flush_out(a, L, nout, -(long long)e, false, spins)) break;
        st_push += (unsigned long long)nout;

        // ---- negative-cycle search once the work looks unbounded --------
        const unsigned long long work = base + e - head0;
        if (work > suspect_after && (base - head0) / walk_stride != work / walk_stride) {
            ++st_walk;
            const unsigned budget = (unsigned)(a.n < (1 << 20) ? a.n + 1 : (1 << 20));
            if (walk_finds_negative_cycle(a, L.u[0], budget)) {
                if (lane == 0) {
                    bq::st_rlx(&q.ctrl->negcycle.v, 1ull);
                    bq::st_rlx(&q.ctrl->abort.v, 1ull);
                }
                break;
            }
        }
    }

    // wave totals -> control block
    if (lane == 0) {
        bq::Ctrl* c = q.ctrl;
        if (st_deq) bq::add_rlx(&c->stats[bq::ST_DEQ].v, st_deq);
        if (st_relax) bq::add_rlx(&c->stats[bq::ST_RELAX].v, st_relax);
        if (st_push) bq::add_rlx(&c->stats[bq::ST_PUSH].v, st_push);
        if (st_fan) bq::add_rlx(&c->stats[bq::ST_FANOUT].v, st_fan);
        if (st_batch) bq::add_rlx(&c->stats[bq::ST_BATCH].v, st_batch);
        if (st_walk) bq::add_rlx(&c->stats[bq::ST_WALK].v, st_walk);
        if (spins) bq::add_rlx(&c->stats[bq::ST_SPIN].v, spins);
        if (st_idle) bq::add_rlx(&c->stats[bq::ST_IDLE].v, st_idle);
        if (st_poll) bq::add_rlx(&c->stats[bq::ST_POLL].v, st_poll);
    }
    // improvements are per lane
    for (int off = 32; off > 0; off >>= 1) st_impr += __shfl_xor(st_impr, off, 64);
    if (lane == 0 && st_impr) bq::add_rlx(&q.ctrl->stats[bq::ST_IMPROVE].v, st_impr);
}

// dist[v] = d, pred[v] = parent (INT64_MAX / -1 when unreached; pred[src] = -1)
__global__ void k_unpack(long long* key, int* pred, int n, int src, unsigned shift) {
    const long long dmax = KEY_INF >> shift;
    const unsigned pmask = (1u << (shift - 1u)) - 1u;
    for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v < n;
         v += (long long)gridDim.x * blockDim.x) {
        const long long k = key[v];
        const long long d = k >> shift;
        const bool reached = d != dmax;
        key[v] = reached ? d : LLONG_MAX;
        if (pred) pred[v] = (reached && v != src) ? (int)(((unsigned long long)k >> 1) & pmask) : -1;
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// host API
// ---------------------------------------------------------------------------
struct sssp_ctx {
    int device;
    int max_n;
    long long max_m;
    uint32_t capacity, logN;
    unsigned long long* slots;
    bq::Ctrl* ctrl;
    unsigned* chunk_owner;
    int* wrange;                  // [2 * INIT_MAX_BLOCKS]
    unsigned long long* trace;    // [4 * TRACE_CAP]
    unsigned long long* h_trace;  // pinned copy
    int trace_n;
    unsigned chunk_log;
    bq::Ctrl* h_ctrl;  // pinned copy of the control block
    hipEvent_t ev0, ev1, evs0, evs1;
    bool dirty;        // queue state must be rebuilt before the next solve
    sssp_stats last;
    int solve_per_cu[3];
};

namespace {

constexpr unsigned DEFAULT_CHUNK_LOG = 10;  // rows longer than 1024 edges are split
constexpr unsigned MIN_CHUNK_LOG = 6;       // smallest row chunk a launch may ask for
constexpr unsigned MAX_CHUNK_LOG = 16;
constexpr int TRACE_CAP = 4096;

bq_status ctx_reset_queue(sssp_ctx* c, hipStream_t s) {
    BQ_HIP_TRY(hipMemsetAsync(c->slots, 0, sizeof(unsigned long long) * c->capacity, s));
    BQ_HIP_TRY(hipMemsetAsync(c->ctrl, 0, sizeof(bq::Ctrl), s));
    c->dirty = false;
    return BQ_OK;
}

Queue ctx_queue(const sssp_ctx* c) {
    Queue q;
    q.slots = c->slots;
    q.ctrl = c->ctrl;
    q.logN = c->logN;
    q.pad = 0;
    q.N = 1ull << c->logN;
    return q;
}

unsigned key_shift(int n) {
    unsigned pb = 0;
    while ((1ull << pb) < (unsigned long long)n + 1ull) ++pb;  // sentinel 2^pb - 1 >= n
    return pb + 1u;
}

int grid_for(int n_items) {
    int g = (n_items + 255) / 256;
    const int cap = 8 * bqh::device_cus();
    if (g > cap) g = cap;
    return g < 1 ? 1 : g;
}

// Default workgroup count when the caller gives none: about one workgroup
// (4 waves) per 16K units of n + m/16, a power of two between 4 and the
// co-resident maximum. More waves than the work can feed only add traffic on
// the queue's hot lines and extra relaxations (labels scanned before they
// settle); sssp_autotune measures instead of guessing.
int default_grid(int n, long long m, int max_grid) {
    const unsigned long long units = (unsigned long long)n + (unsigned long long)m / 16ull;
    int g = 4;
    while ((unsigned long long)g * 2ull * 16384ull <= units && g * 2 <= max_grid) g *= 2;
    return g < max_grid ? g : max_grid;
}

template <int B>
bq_status launch_solve(sssp_ctx* c, const SolveArgs& args, const bqh::Launch& L, hipStream_t s,
                       int slot, int* grid_out) {
    int& per_cu = c->solve_per_cu[slot];
    if (per_cu == 0) {
        BQ_HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_solve<B>, SOLVE_WG, 0));
        if (per_cu < 1) per_cu = 1;
    }
    const int max_grid = per_cu * bqh::device_cus();
    int grid = L.wg_count > 0 ? L.wg_count : default_grid(args.n, args.m, max_grid);
    if (grid > max_grid) grid = max_grid;  // all waves co-resident
    *grid_out = grid;
    hipLaunchKernelGGL(k_solve<B>, dim3(grid), dim3(SOLVE_WG), 0, s, args);
    BQ_HIP_TRY(hipGetLastError());
    return BQ_OK;
}

}  // namespace

extern "C" {

bq_status sssp_ctx_create(int32_t max_n, int64_t max_m, sssp_ctx** out) {
    if (!out || max_n < 1 || max_m < 0) return BQ_EINVAL;
    *out = nullptr;
    sssp_ctx* c = (sssp_ctx*)calloc(1, sizeof(sssp_ctx));
    if (!c) return BQ_ENOMEM;
    BQ_HIP_TRY(hipGetDevice(&c->device));
    c->max_n = max_n;
    c->max_m = max_m;
    c->chunk_log = DEFAULT_CHUNK_LOG;
    // items in the queue: at most n vertices (one per vertex, the q bit) plus
    // chunk items (at most m / C per fan-out generation); capacity
    // 2 * pow2(n + m / C_min), at least 4096
    const unsigned long long need =
        (unsigned long long)max_n + ((unsigned long long)max_m >> MIN_CHUNK_LOG) + 1ull;
    unsigned long long cap = 4096ull;
    while (cap < 2ull * need) cap <<= 1;
    if (cap > (1ull << 31)) {
        free(c);
        return BQ_EINVAL;
    }
    c->capacity = (uint32_t)cap;
    c->logN = bqh::log2_exact(cap);
    const size_t chunks = (size_t)((unsigned long long)max_m >> MIN_CHUNK_LOG) + 1;
    if (hipMalloc(&c->slots, sizeof(unsigned long long) * cap) != hipSuccess ||
        hipMalloc(&c->trace, sizeof(unsigned long long) * 4 * TRACE_CAP) != hipSuccess ||
        hipHostMalloc(&c->h_trace, sizeof(unsigned long long) * 4 * TRACE_CAP,
                      hipHostMallocDefault) != hipSuccess ||
        hipMalloc(&c->ctrl, sizeof(bq::Ctrl)) != hipSuccess ||
        hipMalloc(&c->chunk_owner, sizeof(unsigned) * chunks) != hipSuccess ||
        hipMalloc(&c->wrange, sizeof(int) * 2 * INIT_MAX_BLOCKS) != hipSuccess ||
        hipHostMalloc(&c->h_ctrl, sizeof(bq::Ctrl), hipHostMallocDefault) != hipSuccess) {
        sssp_ctx_destroy(c);
        return BQ_ENOMEM;
    }
    BQ_HIP_TRY(hipEventCreate(&c->ev0));
    BQ_HIP_TRY(hipEventCreate(&c->ev1));
    BQ_HIP_TRY(hipEventCreate(&c->evs0));
    BQ_HIP_TRY(hipEventCreate(&c->evs1));
    bq_status st = ctx_reset_queue(c, nullptr);
    if (st != BQ_OK) {
        sssp_ctx_destroy(c);
        return st;
    }
    BQ_HIP_TRY(hipDeviceSynchronize());
    *out = c;
    return BQ_OK;
}

bq_status sssp_ctx_destroy(sssp_ctx* c) {
    if (!c) return BQ_OK;
    (void)hipDeviceSynchronize();
    if (c->slots) (void)hipFree(c->slots);
    if (c->trace) (void)hipFree(c->trace);
    if (c->h_trace) (void)hipHostFree(c->h_trace);
    if (c->ctrl) (void)hipFree(c->ctrl);
    if (c->chunk_owner) (void)hipFree(c->chunk_owner);
    if (c->wrange) (void)hipFree(c->wrange);
    if (c->h_ctrl) (void)hipHostFree(c->h_ctrl);
    if (c->ev0) (void)hipEventDestroy(c->ev0);
    if (c->ev1) (void)hipEventDestroy(c->ev1);
    if (c->evs0) (void)hipEventDestroy(c->evs0);
    if (c->evs1) (void)hipEventDestroy(c->evs1);
    free(c);
    return BQ_OK;
}

bq_status sssp_autotune(sssp_ctx* c, int32_t n, int64_t m, const int64_t* d_offsets,
                        const int32_t* d_cols, const int32_t* d_w, int32_t src, int64_t* d_dist,
                        const bq_launch* base, int32_t reps, bq_launch* h_best,
                        double* h_best_ms, void* stream) {
    if (!c || !h_best || !h_best_ms || !d_dist) return BQ_EINVAL;
    if (reps < 1) reps = 2;
    bq_launch L = {};
    if (base) L = *base;
    L.flags &= ~(uint32_t)(BQ_F_TRACE | BQ_F_VALIDATE);
    int per_cu = c->solve_per_cu[0];
    if (per_cu == 0) {
        BQ_HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_solve<64>, SOLVE_WG, 0));
        if (per_cu < 1) per_cu = 1;
        c->solve_per_cu[0] = per_cu;
    }
    const int max_grid = per_cu * bqh::device_cus();
    double best = 1e300;
    bq_launch bestL = L;
    auto trial = [&](int wgs, int b, double* out_ms, int chunk = -1) -> bq_status {
        bq_launch t = L;
        t.wg_count = wgs;
        t.ticket_batch = b;
        if (chunk >= 0) t.row_chunk = chunk;
        double tmin = 1e300;
        for (int r = 0; r < reps; ++r) {
            int32_t neg = 0;
            bq_status st = sssp_bf(c, n, m, d_offsets, d_cols, d_w, src, d_dist, nullptr, &neg,
                                   &t, stream);
            if (st != BQ_OK) return st;
            if (c->last.ms < tmin) tmin = c->last.ms;
        }
        *out_ms = tmin;
        if (tmin < best) {
            best = tmin;
            bestL = t;
        }
        return BQ_OK;
    };
    // workgroup count: powers of two upwards until clearly past the minimum
    int best_wgs = 4;
    for (int wgs = 4; wgs <= max_grid; wgs *= 2) {
        double ms = 0;
        bq_status st = trial(wgs, 1, &ms);
        if (st != BQ_OK) return st;
        if (ms <= best) best_wgs = wgs;
        if (ms > 2.0 * best && wgs >= 4 * best_wgs) break;
        if (wgs * 2 > max_grid && wgs != max_grid) {
            st = trial(max_grid, 1, &ms);
            if (st != BQ_OK) return st;
        }
    }
    // ticket batch at the best count and its neighbours
    for (int b = 2; b <= 4; b *= 2) {
        for (int f = -1; f <= 1; ++f) {
            int wgs = f < 0 ? best_wgs / 2 : (f > 0 ? best_wgs * 2 : best_wgs);
            if (wgs < 1 || wgs > max_grid) continue;
            double ms = 0;
            bq_status st = trial(wgs, b, &ms);
            if (st != BQ_OK) return st;
        }
    }
    // row chunk around the default at the best shape so far
    {
        const bq_launch cur = bestL;
        for (int chunk : {256, 4096}) {
            double ms = 0;
            bq_status st = trial(cur.wg_count, cur.ticket_batch, &ms, chunk);
            if (st != BQ_OK) return st;
        }
    }
    *h_best = bestL;
    *h_best_ms = best;
    return BQ_OK;
}

int32_t sssp_last_trace(const sssp_ctx* c, uint64_t* h_out, int32_t cap_samples) {
    if (!c || !h_out || cap_samples < 0) return BQ_EINVAL;
    int k = c->trace_n < cap_samples ? c->trace_n : cap_samples;
    for (int i = 0; i < 4 * k; ++i) h_out[i] = c->h_trace[i];
    return k;
}

bq_status sssp_last_stats(const sssp_ctx* c, sssp_stats* out) {
    if (!c || !out) return BQ_EINVAL;
    *out = c->last;
    return BQ_OK;
}

bq_status sssp_bf(sssp_ctx* c, int32_t n, int64_t m, const int64_t* d_offsets,
                  const int32_t* d_cols, const int32_t* d_w, int32_t src, int64_t* d_dist,
                  int32_t* d_pred, int32_t* h_neg_cycle, const bq_launch* launch, void* stream) {
    if (!c || !d_offsets || !d_dist || !h_neg_cycle) return BQ_EINVAL;
    if (n < 1 || m < 0 || src < 0 || src >= n) return BQ_EINVAL;
    if (m > 0 && (!d_cols || !d_w)) return BQ_EINVAL;
    if (n > c->max_n || m > c->max_m) return BQ_EBUSY;
    unsigned clog = DEFAULT_CHUNK_LOG;
    if (launch && launch->row_chunk > 0) {
        const int rc = launch->row_chunk;
        if (rc & (rc - 1)) return BQ_EINVAL;
        clog = bqh::log2_exact((unsigned long long)rc);
        if (clog < MIN_CHUNK_LOG || clog > MAX_CHUNK_LOG) return BQ_EINVAL;
    }
    // items are vertex ids below n and chunk ids n + j; both must fit 32 bits
    if ((unsigned long long)n + ((unsigned long long)m >> clog) + 1ull >= 0xFFFFFFFFull)
        return BQ_EINVAL;
    hipStream_t s = bqh::as_stream(stream);
    bqh::Launch L = bqh::resolve(launch, 0);
    if (L.batch != 1 && L.batch != 2 && L.batch != 4) return BQ_EINVAL;
    if (c->dirty) {
        bq_status st = ctx_reset_queue(c, s);
        if (st != BQ_OK) return st;
    }
    const Queue q = ctx_queue(c);
    if (L.flags & BQ_F_VALIDATE) {
        BQ_HIP_TRY(hipMemsetAsync(&c->ctrl->aux[3].v, 0, 8, s));
        hipLaunchKernelGGL(k_validate, dim3(grid_for((int)(m > n ? (m > INT_MAX ? INT_MAX : m) : n))),
                           dim3(256), 0, s, (const long long*)d_offsets, (const int*)d_cols, n,
                           (long long)m, c->ctrl);
        BQ_HIP_TRY(hipGetLastError());
        unsigned long long bad = 0;
        BQ_HIP_TRY(hipMemcpyAsync(&bad, &c->ctrl->aux[3].v, 8, hipMemcpyDeviceToHost, s));
        BQ_HIP_TRY(hipStreamSynchronize(s));
        if (bad) return BQ_EINVAL;
    }
    const unsigned shift = key_shift(n);
    SolveArgs a;
    a.q = q;
    a.off = (const long long*)d_offsets;
    a.col = (const int*)d_cols;
    a.w = (const int*)d_w;
    a.key = (long long*)d_dist;
    a.chunk_owner = c->chunk_owner;
    a.wrange = c->wrange;
    a.n = n;
    a.src = src;
    a.m = (long long)m;
    a.shift = shift;
    a.chunk_log = clog;
    a.limit = L.limit;
    a.deadline = 10ull * L.limit;
    a.trace = nullptr;
    a.trace_shift = 0;
    a.trace_cap = TRACE_CAP;
    if (L.flags & BQ_F_TRACE) {
        // about 256 samples per n + m/C items of work
        unsigned long long unit = (unsigned long long)n + ((unsigned long long)m >> clog);
        unsigned sh = 0;
        while ((1ull << (sh + 8)) < unit) ++sh;
        a.trace = c->trace;
        a.trace_shift = sh;
        BQ_HIP_TRY(hipMemsetAsync(c->trace, 0xff, sizeof(unsigned long long) * 4 * TRACE_CAP, s));
    }

    BQ_HIP_TRY(hipEventRecord(c->ev0, s));
    {
        const long long big = m > n ? m : n;
        long long blocks = (big + (long long)INIT_WG * 8 - 1) / ((long long)INIT_WG * 8);
        if (blocks < 1) blocks = 1;
        if (blocks > INIT_MAX_BLOCKS) blocks = INIT_MAX_BLOCKS;
        hipLaunchKernelGGL(k_init, dim3((unsigned)blocks), dim3(INIT_WG), 0, s, q,
                           (long long*)d_dist, n, src, shift, (const int*)d_w, (long long)m,
                           c->wrange);
        BQ_HIP_TRY(hipGetLastError());
    }
    int grid = 0;
    bq_status st;
    BQ_HIP_TRY(hipEventRecord(c->evs0, s));
    switch (L.batch) {
        case 1: st = launch_solve<64>(c, a, L, s, 0, &grid); break;
        case 2: st = launch_solve<128>(c, a, L, s, 1, &grid); break;
        default: st = launch_solve<256>(c, a, L, s, 2, &grid); break;
    }
    if (st != BQ_OK) return st;
    BQ_HIP_TRY(hipEventRecord(c->evs1, s));
    hipLaunchKernelGGL(k_unpack, dim3(grid_for(n)), dim3(256), 0, s, (long long*)d_dist,
                       (int*)d_pred, n, src, shift);
    BQ_HIP_TRY(hipGetLastError());
    BQ_HIP_TRY(hipEventRecord(c->ev1, s));
    BQ_HIP_TRY(hipMemcpyAsync(c->h_ctrl, c->ctrl, sizeof(bq::Ctrl), hipMemcpyDeviceToHost, s));
    c->trace_n = 0;
    if (a.trace) {
        BQ_HIP_TRY(hipMemcpyAsync(c->h_trace, c->trace, sizeof(unsigned long long) * 4 * TRACE_CAP,
                                  hipMemcpyDeviceToHost, s));
        c->trace_n = TRACE_CAP;
    }
    BQ_HIP_TRY(hipStreamSynchronize(s));
    const bq::Ctrl* h = c->h_ctrl;
    float ms = 0.f, sms = 0.f;
    BQ_HIP_TRY(hipEventElapsedTime(&ms, c->ev0, c->ev1));
    BQ_HIP_TRY(hipEventElapsedTime(&sms, c->evs0, c->evs1));
    c->last.dequeued = h->stats[bq::ST_DEQ].v;
    c->last.relaxations = h->stats[bq::ST_RELAX].v;
    c->last.pushes = h->stats[bq::ST_PUSH].v;
    c->last.fanout = h->stats[bq::ST_FANOUT].v;
    c->last.batches = h->stats[bq::ST_BATCH].v;
    c->last.walks = h->stats[bq::ST_WALK].v;
    c->last.improvements = h->stats[bq::ST_IMPROVE].v;
    c->last.idle_polls = h->stats[bq::ST_POLL].v;
    c->last.ticket_spins = h->stats[bq::ST_SPIN].v;
    c->last.ms = ms;
    c->last.solve_ms = sms;
    c->last.grid = grid;
    c->last.wg_size = SOLVE_WG;
    const unsigned long long err = h->error.v;
    const bool neg = h->negcycle.v != 0ull;
    if (err != 0ull || neg || h->abort.v != 0ull) c->dirty = true;  // queue not quiescent
    if (err == bq::ERR_RANGE) return BQ_ERANGE;
    if (err != 0ull) return BQ_ETIMEOUT;
    *h_neg_cycle = neg ? 1 : 0;
    return BQ_OK;
}

}  // extern "C"
