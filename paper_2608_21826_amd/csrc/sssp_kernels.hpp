// Kernels of the single-query launch (init, persistent solver, unpack).
// Kept apart from the host code in sssp.hip so that the device code the
// counter summaries were taken on can be identified by these files alone.
#pragma once
#include <hip/hip_runtime.h>
#include <limits.h>

#include "sssp_device.hpp"

namespace {

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
    // keys in 16-byte stores and weights in 16-byte loads, each after a
    // scalar head up to 16-byte alignment and with a scalar tail (the
    // caller's arrays need only their element alignment)
    {
        const long long head = (((uintptr_t)key & 15u) && n > 0) ? 1 : 0;
        const long long n2 = (n - head) >> 1;
        for (long long v = tid; v < head; v += stride) key[v] = (v == src) ? srckey : KEY_INF;
        longlong2* k2 = (longlong2*)(key + head);
        for (long long i = tid; i < n2; i += stride) {
            const long long v0 = head + 2 * i;
            longlong2 x;
            x.x = (v0 == src) ? srckey : KEY_INF;
            x.y = (v0 + 1 == src) ? srckey : KEY_INF;
            k2[i] = x;
        }
        for (long long v = head + 2 * n2 + tid; v < n; v += stride)
            key[v] = (v == src) ? srckey : KEY_INF;
    }
    int lo = INT_MAX, hi = INT_MIN;
    {
        long long wh = (long long)(((16u - ((uintptr_t)w & 15u)) & 15u) >> 2);
        if (wh > m) wh = m;
        const long long m4 = (m - wh) >> 2;
        for (long long e = tid; e < wh; e += stride) {
            const int x = w[e];
            lo = x < lo ? x : lo;
            hi = x > hi ? x : hi;
        }
        const int4* w4 = (const int4*)(w + wh);
        for (long long i = tid; i < m4; i += stride) {
            const int4 x = w4[i];
            const int l01 = x.x < x.y ? x.x : x.y, l23 = x.z < x.w ? x.z : x.w;
            const int h01 = x.x > x.y ? x.x : x.y, h23 = x.z > x.w ? x.z : x.w;
            const int l = l01 < l23 ? l01 : l23, h = h01 > h23 ? h01 : h23;
            lo = l < lo ? l : lo;
            hi = h > hi ? h : hi;
        }
        for (long long e = wh + 4 * m4 + tid; e < m; e += stride) {
            const int x = w[e];
            lo = x < lo ? x : lo;
            hi = x > hi ? x : hi;
        }
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
    c->aux[1].v = (unsigned long long)LLONG_MIN;  // near / far threshold (buckets)
    c->busy.v = 0ull;
    for (unsigned sg = 0; sg < MAX_Q; ++sg)        // dequeue positions at start
        q.ctrl[sg].aux[2].v = q.ctrl[sg].head.v;
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

template <int B, int UU>
__device__ __forceinline__ void solve_kernel_body(const SolveArgs& a) {
    __shared__ WaveLds<B> lds[WAVES_PER_WG_ONE];
    __shared__ WgShared S;
    WaveLds<B>& L = lds[threadIdx.x >> 6];
    const int wid = (int)(threadIdx.x >> 6);
    if (threadIdx.x == 0) {
        S.poller = -1;
        S.wake = 0u;
        S.done = 0;
    }
    __syncthreads();
    WaveStats st{};
    solve_instance<B, true, UU>(a, L, S, wid, st);
    flush_stats(a.q.ctrl->stats, st);
}

template <int B>
__global__ __launch_bounds__(SOLVE_WG_ONE, SSSP_MIN_WAVES) void k_solve(SolveArgs a) {
    solve_kernel_body<B, U>(a);
}

// the same solver with SHORT_ROW_UNROLL edges per lane per scan step, for
// graphs whose rows are short on average (see launch_solve)
template <int B, int UU>
__global__ __launch_bounds__(SOLVE_WG_ONE, SSSP_MIN_WAVES) void k_solve_short(SolveArgs a) {
    solve_kernel_body<B, UU>(a);
}

// dist[v] = d, pred[v] = parent (INT64_MAX / -1 when unreached; pred[src] = -1;
// INT64_MIN / -1 for minus infinity)
__global__ void k_unpack(long long* key, int* pred, int n, int src, unsigned shift) {
    const long long dmax = KEY_INF >> shift;
    const unsigned pmask = (1u << (shift - 1u)) - 1u;
    for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v < n;
         v += (long long)gridDim.x * blockDim.x) {
        const long long k = key[v];
        if (is_neg_key(k)) {  // minus infinity (marking mode)
            key[v] = LLONG_MIN;
            if (pred) pred[v] = -1;
            continue;
        }
        const long long d = k >> shift;
        const bool reached = d != dmax;
        key[v] = reached ? d : LLONG_MAX;
        if (pred) pred[v] = (reached && v != src) ? (int)(((unsigned long long)k >> 1) & pmask) : -1;
    }
}

}  // namespace
