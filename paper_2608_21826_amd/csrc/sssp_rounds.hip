// Round-based Bellman-Ford over an edge queue: the paper's own single-GPU
// form (Section III.C) and Alg. 3 run on one processing element.
//
// The Broker Queue holds edges. A round enqueues every edge id once and the
// same kernel's waves dequeue them concurrently and relax them:
//   d[v] <- min(d[v], d[u] + w)   when d[u] is finite          (Alg. 3)
// counting the relaxations that lowered d[v] in a per-round `changes`
// counter. After round i: no change ends the solve (early exit); a change in
// round n-1 (the n-th round) proves a negative cycle reachable from the
// source. Distances are the caller's plain int64 array (infinity INT64_MAX);
// the lowering is an atomicMin, so no update is lost.
//
// Why the rounds give the same answer as the sequential rounds of one
// processing element: a relaxation reads d[u] at some moment of the round,
// never above its value at the round's start, so after round i every d[v] is
// at most the weight of the best walk of i+1 edges, as in the sequential
// form. With no negative cycle nothing changes once the n-1 rounds have
// fixed every shortest path, so round n-1 sees no change; with one, some
// distance falls in every round.
//
// Launch structure (host loop, as in Alg. 3's loop over i): per round one
// persistent kernel (all waves co-resident) and one single-lane check kernel
// that reads `changes`, decides, and resets it. Rounds are issued in groups
// without a host round trip; a round issued after the solve has ended sees
// the done word and returns at once. The host synchronizes once per group.
#include <hip/hip_runtime.h>
#include <limits.h>
#include <stdlib.h>
#include <time.h>

#include "bq_device.hpp"
#include "csr_device.hpp"
#include "host_common.hpp"

namespace {

using bq::Queue;

constexpr long long DINF = LLONG_MAX;
constexpr int PREP_WG = 256;
constexpr int ROUND_MAX_WG = 1024;

// control words used here (bq::Ctrl): head / tail / count are the queue's;
// aux[0] changes in the current round, aux[1] done, aux[2] dequeue position
// where the current round's items start, aux[3] CSR defect, aux[4] max |w|,
// aux[5] rounds run, stats[ST_IMPROVE] changes over all rounds,
// stats[ST_SPIN] ticket waits.
enum : int { A_CHANGES = 0, A_DONE = 1, A_BASE = 2, A_BAD = 3, A_WMAX = 4, A_ROUNDS = 5 };

struct RoundArgs {
    Queue q;
    const int* esrc;  // [m] source vertex of each edge, built from the CSR
    const int* col;   // [m]
    const int* w;     // [m]
    long long* dist;  // [n]
    long long m;
    int n;
    unsigned items;  // edge ids per wave queue operation (64 * b)
    unsigned bwd;    // dequeue broker policy: 0 Broker Queue, 1 BWD
    unsigned pad;
    unsigned long long limit;  // one wait, ticks of the 100 MHz clock
};

// Control words of a new solve; the queue itself is quiescent (head == tail,
// count == 0) and keeps its positions and tickets.
__global__ void k_reset(bq::Ctrl* c) {
    if (threadIdx.x != 0) return;
    c->abort.v = 0ull;
    c->error.v = 0ull;
    c->negcycle.v = 0ull;
    c->aux[A_CHANGES].v = 0ull;
    c->aux[A_DONE].v = 0ull;
    c->aux[A_BASE].v = c->head.v;
    c->aux[A_WMAX].v = 0ull;
    c->aux[A_ROUNDS].v = 0ull;
    for (int i = 0; i < bq::ST_N; ++i) c->stats[i].v = 0ull;
}

// Distances (d[src] = 0, otherwise infinity) and the largest |w|.
__global__ __launch_bounds__(PREP_WG) void k_prep(const int* w, int n, long long m, int src,
                                                  long long* dist, bq::Ctrl* ctrl) {
    const long long tid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long v = tid; v < n; v += stride) dist[v] = v == src ? 0ll : DINF;
    unsigned long long wmax = 0;
    for (long long e = tid; e < m; e += stride) {
        const long long x = w[e];
        const unsigned long long a = (unsigned long long)(x < 0 ? -x : x);
        wmax = a > wmax ? a : wmax;
    }
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long y = __shfl_xor(wmax, o, 64);
        wmax = y > wmax ? y : wmax;
    }
    if (bq::lane_id() == 0 && wmax)
        __hip_atomic_fetch_max(&ctrl->aux[A_WMAX].v, wmax, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
}

// Edge-source array esrc[e] = the row holding edge e. Waves take ranges of
// SRC_RANGE edges, so a hub row is shared out like any other edges. A range
// starts in the row found by a binary search over the offsets. In each step
// of 64 edges the lanes hold the ends of the next 64 rows (as 32-bit
// distances from the range start) and every lane finds its row by a binary
// search over them; the window slides by 64 rows while some edge lies
// beyond it (runs of empty rows).
constexpr long long SRC_RANGE = 4096;

__global__ __launch_bounds__(PREP_WG) void k_edge_src(const long long* off, int n, long long m,
                                                      int* esrc) {
    const int lane = bq::lane_id();
    const long long wave = ((long long)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const long long waves = ((long long)gridDim.x * blockDim.x) >> 6;
    for (long long E = wave * SRC_RANGE; E < m; E += waves * SRC_RANGE) {
        const long long Eend = E + SRC_RANGE < m ? E + SRC_RANGE : m;
        // largest r with off[r] <= E (off[0] = 0 <= E < m = off[n])
        long long r = 0;
        if (lane == 0) {
            long long lo = 0, hi = n;
            while (hi - lo > 1) {
                const long long mid = (lo + hi) >> 1;
                if (off[mid] <= E) lo = mid;
                else hi = mid;
            }
            r = lo;
        }
        r = (long long)bq::bcast64((unsigned long long)r);
        for (long long e0 = E; e0 < Eend; e0 += 64) {
            const long long e = e0 + lane;
            const bool act = e < Eend;
            const int x = (int)(e - E);
            long long row = -1;
            bool todo = act;
            while (__any(todo)) {
                const long long j = r + 1 + lane;
                const long long d = (j <= n ? off[j] : LLONG_MAX) - E;
                const int rel = d > INT_MAX ? INT_MAX : (int)d;
                // rows r .. r+cnt-1 end at or before e: e lies in row r+cnt
                int cnt = 0;
#pragma unroll
                for (int step = 32; step > 0; step >>= 1) {
                    const int v = __shfl(rel, cnt + step - 1, 64);
                    if (v <= x) cnt += step;
                }
                if (__shfl(rel, 63, 64) <= x) cnt = 64;  // past this window
                if (todo && cnt < 64) {
                    row = r + cnt;
                    todo = false;
                }
                if (__any(todo)) r += 64;
            }
            if (act) esrc[e] = (int)row;
            // the next step starts in the row of this step's last edge
            const int last = (int)((Eend - e0 < 64 ? Eend - e0 : 64) - 1);
            r = __shfl(row, last, 64);
        }
    }
}

// One round: enqueue every edge id (grid-stride chunks of `items`), then
// dequeue and relax until the round's m items have all been taken.
__global__ __launch_bounds__(ROUND_MAX_WG) void k_round(RoundArgs a) {
    const Queue& q = a.q;
    bq::Ctrl* c = q.ctrl;
    if (bq::bcast64(bq::ld_rlx(&c->aux[A_DONE].v)) != 0ull) return;
    const int lane = bq::lane_id();
    const long long waves = ((long long)gridDim.x * blockDim.x) >> 6;
    const long long gw = ((long long)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const long long K = a.items;
    unsigned long long spins = 0;

    // ---- ENQUEUE: ENSURE on count, positions from tail, PUT_DATA -------
    for (long long c0 = gw * K; c0 < a.m; c0 += waves * K) {
        const unsigned cnt = (unsigned)(a.m - c0 < K ? a.m - c0 : K);
        unsigned long long base = 0;
        unsigned ok = 0;
        if (lane == 0) {
            ok = bq::reserve_enqueue(q, cnt);  // capacity >= m: never short
            if (ok == cnt) base = bq::add_rlx(&c->tail.v, (unsigned long long)cnt);
        }
        ok = bq::bcast32(ok);
        if (ok != cnt) {
            if (lane == 0) bq::raise_error(q, bq::ERR_FULL);
            return;
        }
        base = bq::bcast64(base);
        for (unsigned i0 = 0; i0 < cnt; i0 += 64) {
            const unsigned i = i0 + lane;
            if (!bq::put_slots(q, i < cnt, base + i, (unsigned)(c0 + i), a.limit, spins)) return;
        }
    }

    // ---- DEQUEUE and relax ---------------------------------------------
    const unsigned long long end = bq::bcast64(bq::ld_rlx(&c->aux[A_BASE].v)) +
                                   (unsigned long long)a.m;
    bool optimistic = true;
    // After a failed take a wave takes again only once the count shows
    // items: a BWD take is blind, and a crowd of idle waves taking blindly
    // would hold the count below zero and starve each other.
    bool look = false;
    bq::Watch idle;
    idle.arm(a.limit);
    int level = 0;
    while (true) {
        unsigned e = 0;
        unsigned long long base = 0;
        if (lane == 0 && (!look || bq::ld_rlx((BQ_GLOBAL const long long*)(&c->count.v)) > 0)) {
            e = bq::ensure_dequeue(q, (unsigned)K, optimistic, a.bwd != 0);
            if (e) base = bq::add_rlx(&c->head.v, (unsigned long long)e);
        }
        e = bq::bcast32(e);
        optimistic = e == (unsigned)K;
        look = e == 0;
        if (e == 0) {
            // the round is over for this wave once every item has a taker
            if (bq::bcast64(bq::ld_rlx(&c->head.v)) >= end) break;
            if (bq::aborted(q)) break;
            if (idle.expired()) {
                if (lane == 0) bq::raise_error(q, bq::ERR_TIMEOUT);
                break;
            }
            bq::idle_backoff(level < 6 ? level++ : level, 64u);
            continue;
        }
        level = 0;
        idle.arm(a.limit);
        base = bq::bcast64(base);
        unsigned improved = 0;
        for (unsigned i0 = 0; i0 < e; i0 += 64) {
            const unsigned i = i0 + lane;
            unsigned id = 0;
            if (!bq::read_slots(q, i < e, base + i, id, a.limit, spins)) {
                i0 = e;  // aborted: leave with the wave
                break;
            }
            bool lower = false;
            if (i < e) {
                const int u = a.esrc[id], v = a.col[id];
                const long long du = bq::ld_rlx(&a.dist[u]);
                if (du != DINF) {
                    const long long cand = du + (long long)a.w[id];
                    if (cand < bq::ld_rlx(&a.dist[v])) {
                        const long long old = __hip_atomic_fetch_min(
                            &a.dist[v], cand, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        lower = cand < old;
                    }
                }
            }
            improved += (unsigned)__popcll(bq::ballot(lower));
        }
        if (lane == 0 && improved)
            bq::add_rlx(&c->aux[A_CHANGES].v, (unsigned long long)improved);
        if (bq::aborted(q)) break;
    }
    if (lane == 0 && spins) bq::add_rlx(&c->stats[bq::ST_SPIN].v, spins);
}

// End of round i (Alg. 3's test after each pass): no change -> done;
// a change in round n-1 -> negative cycle. Before the first decision, the
// range precondition: after n rounds |d| <= n * m * max|w|, which must stay
// below 2^62 so that no d[u] + w overflows.
__global__ void k_check(bq::Ctrl* c, long long round, int n, long long m) {
    if (threadIdx.x != 0 || c->aux[A_DONE].v != 0ull) return;
    if (c->error.v != 0ull || c->abort.v != 0ull) {
        c->aux[A_DONE].v = 1ull;
        return;
    }
    if (round == 0) {
        const double bound = ((double)n + 1.0) * ((double)m + 1.0) * (double)c->aux[A_WMAX].v;
        if (bound >= 4611686018427387904.0) {  // 2^62
            c->error.v = (unsigned long long)bq::ERR_RANGE;
            c->aux[A_DONE].v = 1ull;
            return;
        }
    }
    const unsigned long long changes = c->aux[A_CHANGES].v;
    c->aux[A_CHANGES].v = 0ull;
    c->stats[bq::ST_IMPROVE].v += changes;
    c->aux[A_ROUNDS].v = (unsigned long long)round + 1ull;
    c->aux[A_BASE].v += (unsigned long long)m;
    if (changes == 0ull) {
        c->aux[A_DONE].v = 1ull;
    } else if (round == (long long)n - 1) {
        c->negcycle.v = 1ull;
        c->aux[A_DONE].v = 1ull;
    }
}

// pred[v] = smallest u over edges (u, v, w) with d[u] finite and
// d[u] + w == d[v]; -1 for the source and unreached vertices.
__global__ void k_pred_init(int* pred, int n) {
    for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v < n;
         v += (long long)gridDim.x * blockDim.x)
        pred[v] = INT_MAX;
}

__global__ void k_pred_edges(const int* esrc, const int* col, const int* w, const long long* dist,
                             int* pred, int src, long long m) {
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < m;
         e += (long long)gridDim.x * blockDim.x) {
        const int u = esrc[e], v = col[e];
        const long long du = dist[u];
        if (du != DINF && du != LLONG_MIN && v != src && du + (long long)w[e] == dist[v])
            atomicMin(&pred[v], u);
    }
}

__global__ void k_pred_fix(int* pred, int n) {
    for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v < n;
         v += (long long)gridDim.x * blockDim.x)
        if (pred[v] == INT_MAX) pred[v] = -1;
}

// Minus-infinity marking (flag BQ_F_NEGINF), after the rounds proved a
// negative cycle. The labels are then at least n-1 rounds old: exact for
// every vertex no negative cycle reaches, never below the true distance, and
// finite on every reached vertex. So an edge that still lowers its target
// marks a vertex that a negative cycle reaches, and every negative cycle the
// source reaches has such an edge (the slacks round the cycle sum to its
// weight). The marks are then spread along edges until a pass adds none.
__global__ void k_mark_relaxable(const int* esrc, const int* col, const int* w,
                                 const long long* dist, unsigned* mark, long long m) {
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < m;
         e += (long long)gridDim.x * blockDim.x) {
        const long long du = dist[esrc[e]];
        const int v = col[e];
        if (du != DINF && du + (long long)w[e] < dist[v]) mark[v] = 1u;
    }
}

__global__ void k_mark_spread(const int* esrc, const int* col, unsigned* mark, long long m,
                              bq::Ctrl* c) {
    if (bq::bcast64(bq::ld_rlx(&c->aux[A_DONE].v)) != 0ull) return;
    unsigned grew = 0;
    for (long long e0 = (long long)blockIdx.x * blockDim.x; e0 < m;
         e0 += (long long)gridDim.x * blockDim.x) {
        const long long e = e0 + threadIdx.x;
        bool g = false;
        if (e < m && bq::ld_rlx(&mark[esrc[e]]) != 0u) {
            const int v = col[e];
            g = bq::ld_rlx(&mark[v]) == 0u;
            if (g) bq::st_rlx(&mark[v], 1u);
        }
        grew += (unsigned)__popcll(bq::ballot(g));
    }
    if (bq::lane_id() == 0 && grew) bq::add_rlx(&c->aux[A_CHANGES].v, (unsigned long long)grew);
}

__global__ void k_mark_check(bq::Ctrl* c) {
    if (threadIdx.x != 0 || c->aux[A_DONE].v != 0ull) return;
    if (c->aux[A_CHANGES].v == 0ull) c->aux[A_DONE].v = 1ull;
    c->aux[A_CHANGES].v = 0ull;
}

__global__ void k_mark_apply(long long* dist, const unsigned* mark, int n) {
    for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v < n;
         v += (long long)gridDim.x * blockDim.x)
        if (mark[v]) dist[v] = LLONG_MIN;
}

__global__ void k_mark_reset(bq::Ctrl* c) {
    if (threadIdx.x != 0) return;
    c->aux[A_DONE].v = 0ull;
    c->aux[A_CHANGES].v = 0ull;
}

int grid_for(long long items) {
    long long g = (items + 255) / 256;
    const long long cap = 8ll * bqh::device_cus();
    if (g > cap) g = cap;
    return g < 1 ? 1 : (int)g;
}

}  // namespace

struct sssp_rounds_ctx {
    int device;
    int max_n;
    long long max_m;
    uint32_t capacity, logN;
    unsigned long long* slots;
    bq::Ctrl* ctrl;
    int* esrc;
    unsigned* mark;    // [max_n] minus-infinity marks
    bq::Ctrl* h_ctrl;  // pinned
    hipEvent_t ev0, ev1, evs0, evs1;
    bool dirty;
    int per_cu[5];  // occupancy of k_round at wg_size 64 << i
    sssp_rounds_stats last;
};

namespace {

bq_status rounds_reset_queue(sssp_rounds_ctx* c, hipStream_t s) {
    BQ_HIP_TRY(hipMemsetAsync(c->slots, 0, sizeof(unsigned long long) * c->capacity, s));
    BQ_HIP_TRY(hipMemsetAsync(c->ctrl, 0, sizeof(bq::Ctrl), s));
    c->dirty = false;
    return BQ_OK;
}

double host_seconds() {
    timespec t;
    clock_gettime(CLOCK_MONOTONIC, &t);
    return (double)t.tv_sec + 1e-9 * (double)t.tv_nsec;
}

}  // namespace

extern "C" {

bq_status sssp_rounds_create(int32_t max_n, int64_t max_m, sssp_rounds_ctx** out) {
    if (!out || max_n < 1 || max_m < 0) return BQ_EINVAL;
    *out = nullptr;
    // the queue holds one round's edges: capacity pow2 >= m, at least 4096;
    // edge ids travel as 32-bit payloads
    unsigned long long cap = 4096ull;
    while (cap < (unsigned long long)max_m) cap <<= 1;
    if (cap > (1ull << 31)) return BQ_EINVAL;
    sssp_rounds_ctx* c = (sssp_rounds_ctx*)calloc(1, sizeof(sssp_rounds_ctx));
    if (!c) return BQ_ENOMEM;
    BQ_HIP_TRY(hipGetDevice(&c->device));
    c->max_n = max_n;
    c->max_m = max_m;
    c->capacity = (uint32_t)cap;
    c->logN = bqh::log2_exact(cap);
    const size_t me = (size_t)(max_m > 0 ? max_m : 1);
    if (hipMalloc(&c->slots, sizeof(unsigned long long) * cap) != hipSuccess ||
        hipMalloc(&c->ctrl, sizeof(bq::Ctrl)) != hipSuccess ||
        hipMalloc(&c->esrc, sizeof(int) * me) != hipSuccess ||
        hipMalloc(&c->mark, sizeof(unsigned) * (size_t)max_n) != hipSuccess ||
        hipHostMalloc(&c->h_ctrl, sizeof(bq::Ctrl), hipHostMallocDefault) != hipSuccess ||
        hipEventCreate(&c->ev0) != hipSuccess || hipEventCreate(&c->ev1) != hipSuccess ||
        hipEventCreate(&c->evs0) != hipSuccess || hipEventCreate(&c->evs1) != hipSuccess) {
        sssp_rounds_destroy(c);
        return BQ_ENOMEM;
    }
    bq_status st = rounds_reset_queue(c, nullptr);
    if (st == BQ_OK && hipDeviceSynchronize() != hipSuccess) st = BQ_EHIP;
    if (st != BQ_OK) {
        sssp_rounds_destroy(c);
        return st;
    }
    *out = c;
    return BQ_OK;
}

bq_status sssp_rounds_destroy(sssp_rounds_ctx* c) {
    if (!c) return BQ_OK;
    (void)hipDeviceSynchronize();
    if (c->slots) (void)hipFree(c->slots);
    if (c->ctrl) (void)hipFree(c->ctrl);
    if (c->esrc) (void)hipFree(c->esrc);
    if (c->mark) (void)hipFree(c->mark);
    if (c->h_ctrl) (void)hipHostFree(c->h_ctrl);
    if (c->ev0) (void)hipEventDestroy(c->ev0);
    if (c->ev1) (void)hipEventDestroy(c->ev1);
    if (c->evs0) (void)hipEventDestroy(c->evs0);
    if (c->evs1) (void)hipEventDestroy(c->evs1);
    free(c);
    return BQ_OK;
}

bq_status sssp_rounds_last_stats(const sssp_rounds_ctx* c, sssp_rounds_stats* out) {
    if (!c || !out) return BQ_EINVAL;
    *out = c->last;
    return BQ_OK;
}

bq_status sssp_bf_rounds(sssp_rounds_ctx* c, int32_t n, int64_t m, const int64_t* d_offsets,
                         const int32_t* d_cols, const int32_t* d_w, int32_t src, int64_t* d_dist,
                         int32_t* d_pred, int32_t* h_neg_cycle, const bq_launch* launch,
                         void* stream) {
    if (!c || !d_offsets || !d_dist || !h_neg_cycle) return BQ_EINVAL;
    if (n < 1 || m < 0 || src < 0 || src >= n) return BQ_EINVAL;
    if (m > 0 && (!d_cols || !d_w)) return BQ_EINVAL;
    if (n > c->max_n || m > c->max_m) return BQ_EBUSY;
    hipStream_t s = bqh::as_stream(stream);
    bqh::Launch L = bqh::resolve(launch, 0);
    if (!launch || launch->ticket_batch <= 0) L.batch = 16;
    if (L.batch < 1 || L.batch > 64) return BQ_EINVAL;
    int wsi = -1;
    for (int i = 0; i < 5; ++i)
        if (L.wg_size == (64 << i)) wsi = i;
    if (wsi < 0) return BQ_EINVAL;
    if (c->dirty) {
        bq_status st = rounds_reset_queue(c, s);
        if (st != BQ_OK) return st;
    }
    if (L.flags & BQ_F_VALIDATE) {
        BQ_HIP_TRY(hipMemsetAsync(&c->ctrl->aux[A_BAD].v, 0, 8, s));
        hipLaunchKernelGGL(k_validate_csr, dim3(grid_for(m > n ? m : n)), dim3(256), 0, s,
                           (const long long*)d_offsets, (const int*)d_cols, n, (long long)m,
                           &c->ctrl->aux[A_BAD].v);
        BQ_HIP_TRY(hipGetLastError());
        unsigned long long bad = 0;
        BQ_HIP_TRY(hipMemcpyAsync(&bad, &c->ctrl->aux[A_BAD].v, 8, hipMemcpyDeviceToHost, s));
        BQ_HIP_TRY(hipStreamSynchronize(s));
        if (bad) return BQ_EINVAL;
    }
    int& per_cu = c->per_cu[wsi];
    if (per_cu == 0) {
        BQ_HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_round, L.wg_size, 0));
        if (per_cu < 1) per_cu = 1;
    }
    const int max_grid = per_cu * bqh::device_cus();
    int grid = L.wg_count > 0 ? L.wg_count : 2 * bqh::device_cus();
    if (grid > max_grid) grid = max_grid;  // waits need every wave resident

    RoundArgs a;
    a.q.slots = (decltype(a.q.slots))c->slots;
    a.q.ctrl = (decltype(a.q.ctrl))c->ctrl;
    a.q.sig = (decltype(a.q.sig))c->ctrl;
    a.q.logN = c->logN;
    a.q.pad = 0;
    a.q.N = 1ull << c->logN;
    a.esrc = c->esrc;
    a.col = (const int*)d_cols;
    a.w = (const int*)d_w;
    a.dist = (long long*)d_dist;
    a.m = (long long)m;
    a.n = n;
    a.items = 64u * (unsigned)L.batch;
    a.bwd = (L.flags & BQ_F_BWD) ? 1u : 0u;
    a.pad = 0;
    a.limit = L.limit;
    const double deadline_s = 10.0 * (double)L.limit * 1e-8;  // limit is in 10 ns ticks

    BQ_HIP_TRY(hipEventRecord(c->ev0, s));
    hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, s, c->ctrl);
    BQ_HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_prep, dim3(grid_for(m > n ? m : n)), dim3(PREP_WG), 0, s,
                       (const int*)d_w, n, (long long)m, src, (long long*)d_dist, c->ctrl);
    BQ_HIP_TRY(hipGetLastError());
    if (m > 0) {
        // one wave per range of SRC_RANGE edges, 4 waves per workgroup
        const long long ranges = ((long long)m + SRC_RANGE - 1) / SRC_RANGE;
        const long long cap = 8ll * bqh::device_cus();
        long long blocks = (ranges + 3) / 4;
        if (blocks > cap) blocks = cap;
        hipLaunchKernelGGL(k_edge_src, dim3((unsigned)blocks), dim3(PREP_WG), 0, s,
                           (const long long*)d_offsets, n, (long long)m, c->esrc);
        BQ_HIP_TRY(hipGetLastError());
    }
    BQ_HIP_TRY(hipEventRecord(c->evs0, s));
    const double t0 = host_seconds();
    long long round = 0, group = 4;
    bool timed_out = false;
    while (round < n) {
        const long long stop = round + group < (long long)n ? round + group : (long long)n;
        for (; round < stop; ++round) {
            hipLaunchKernelGGL(k_round, dim3(grid), dim3(L.wg_size), 0, s, a);
            BQ_HIP_TRY(hipGetLastError());
            hipLaunchKernelGGL(k_check, dim3(1), dim3(64), 0, s, c->ctrl, round, n, (long long)m);
            BQ_HIP_TRY(hipGetLastError());
        }
        BQ_HIP_TRY(hipMemcpyAsync(c->h_ctrl, c->ctrl, sizeof(bq::Ctrl), hipMemcpyDeviceToHost, s));
        BQ_HIP_TRY(hipStreamSynchronize(s));
        if (c->h_ctrl->aux[A_DONE].v != 0ull) break;
        if (host_seconds() - t0 > deadline_s) {
            timed_out = true;
            break;
        }
        if (group < 256) group *= 2;
    }
    BQ_HIP_TRY(hipEventRecord(c->evs1, s));
    BQ_HIP_TRY(hipMemcpyAsync(c->h_ctrl, c->ctrl, sizeof(bq::Ctrl), hipMemcpyDeviceToHost, s));
    BQ_HIP_TRY(hipStreamSynchronize(s));
    const bq::Ctrl* h = c->h_ctrl;
    const unsigned long long err = h->error.v;
    const bool neg = h->negcycle.v != 0ull;
    if (err != 0ull) c->dirty = true;  // a wave may have left mid-operation
    const bool neginf = neg && !err && !timed_out && (L.flags & BQ_F_NEGINF);
    if (neginf) {
        BQ_HIP_TRY(hipMemsetAsync(c->mark, 0, sizeof(unsigned) * (size_t)n, s));
        hipLaunchKernelGGL(k_mark_relaxable, dim3(grid_for(m)), dim3(256), 0, s, c->esrc,
                           (const int*)d_cols, (const int*)d_w, (const long long*)d_dist, c->mark,
                           (long long)m);
        BQ_HIP_TRY(hipGetLastError());
        hipLaunchKernelGGL(k_mark_reset, dim3(1), dim3(64), 0, s, c->ctrl);
        BQ_HIP_TRY(hipGetLastError());
        // at most n passes; issued in growing groups like the rounds
        long long pass = 0, grp = 4;
        while (pass < n) {
            const long long stop = pass + grp < (long long)n ? pass + grp : (long long)n;
            for (; pass < stop; ++pass) {
                hipLaunchKernelGGL(k_mark_spread, dim3(grid_for(m)), dim3(256), 0, s, c->esrc,
                                   (const int*)d_cols, c->mark, (long long)m, c->ctrl);
                BQ_HIP_TRY(hipGetLastError());
                hipLaunchKernelGGL(k_mark_check, dim3(1), dim3(64), 0, s, c->ctrl);
                BQ_HIP_TRY(hipGetLastError());
            }
            unsigned long long done = 0;
            BQ_HIP_TRY(hipMemcpyAsync(&done, &c->ctrl->aux[A_DONE].v, 8, hipMemcpyDeviceToHost, s));
            BQ_HIP_TRY(hipStreamSynchronize(s));
            if (done) break;
            if (grp < 256) grp *= 2;
        }
        hipLaunchKernelGGL(k_mark_apply, dim3(grid_for(n)), dim3(256), 0, s, (long long*)d_dist,
                           c->mark, n);
        BQ_HIP_TRY(hipGetLastError());
    }
    if (!err && (!neg || neginf) && !timed_out && d_pred) {
        hipLaunchKernelGGL(k_pred_init, dim3(grid_for(n)), dim3(256), 0, s, (int*)d_pred, n);
        BQ_HIP_TRY(hipGetLastError());
        hipLaunchKernelGGL(k_pred_edges, dim3(grid_for(m)), dim3(256), 0, s, c->esrc,
                           (const int*)d_cols, (const int*)d_w, (const long long*)d_dist,
                           (int*)d_pred, src, (long long)m);
        BQ_HIP_TRY(hipGetLastError());
        hipLaunchKernelGGL(k_pred_fix, dim3(grid_for(n)), dim3(256), 0, s, (int*)d_pred, n);
        BQ_HIP_TRY(hipGetLastError());
    }
    BQ_HIP_TRY(hipEventRecord(c->ev1, s));
    BQ_HIP_TRY(hipEventSynchronize(c->ev1));
    float ms = 0.f, sms = 0.f;
    BQ_HIP_TRY(hipEventElapsedTime(&ms, c->ev0, c->ev1));
    BQ_HIP_TRY(hipEventElapsedTime(&sms, c->evs0, c->evs1));
    c->last.rounds = h->aux[A_ROUNDS].v;
    c->last.changes = h->stats[bq::ST_IMPROVE].v;
    c->last.relaxations = h->aux[A_ROUNDS].v * (unsigned long long)m;
    c->last.ticket_spins = h->stats[bq::ST_SPIN].v;
    c->last.ms = ms;
    c->last.solve_ms = sms;
    c->last.grid = grid;
    c->last.wg_size = L.wg_size;
    if (err == bq::ERR_RANGE) return BQ_ERANGE;
    if (err == bq::ERR_FULL) return BQ_EOVERFLOW;
    if (err != 0ull || timed_out) return BQ_ETIMEOUT;
    *h_neg_cycle = neg ? 1 : 0;
    return BQ_OK;
}

}  // extern "C"
