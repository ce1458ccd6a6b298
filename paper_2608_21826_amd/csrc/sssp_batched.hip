// Batched form: many SSSP queries (different graphs and sources, uneven
// sizes) in one persistent launch, each query with its own Broker Queue.
//
// Three kernels, the same for any batch of a given count, so the sequence
// can be captured once in a hipGraph and replayed:
//  k_binit   - per "unit" (a slice of one query's vertices and edges): keys,
//              weight-range partials; a query's first unit also resets its
//              control block and enqueues its source
//  k_bsolve  - persistent workgroups claim queries from claim lists (queries
//              sorted by size, each listed in proportion to its work, so big
//              queries get several workgroups) and, when their list runs out,
//              join an unfinished query; each runs the solver loop of the
//              single-query launch on that query's queue. There is one list
//              per XCD: a query whose share fits one XCD's workgroups is
//              listed on one list only, so its keys are cached in one L2
//              instead of being spread over all eight
//  k_bunpack - per unit: distances and predecessors; per query: the result
//              flags
#include <hip/hip_runtime.h>
#include <limits.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <tuple>
#include <utility>
#include <vector>

#include "host_common.hpp"
#include "sssp_device.hpp"

namespace {

constexpr unsigned BDEFAULT_CHUNK_LOG = 10;
constexpr unsigned BMIN_CHUNK_LOG = 6;
constexpr unsigned BMAX_CHUNK_LOG = 16;
constexpr long long UNIT = 65536;  // vertices or edges per init/unpack unit
constexpr int BINIT_WG = 256;

struct InstDesc {
    SolveArgs a;
    long long* dist;  // the caller's output (a.key itself unless the key layout is remapped)
    int* pred;
    int orig;        // index in the caller's array
    int unit_begin;  // units [unit_begin, unit_end) belong to this query
    int unit_end;
    int pad;
};

struct Unit {
    int inst;
    int pad;
    long long v0, v1, e0, e1;
};

// Degree-class key layout of a graph that several queries of the batch share
// (see remap in sssp_bf_batched_start): key positions are ordered by class of
// out-degree, highest first, then by vertex id, so that the keys of the
// vertices most edges point at share few cache lines and stay in L2.
constexpr int RM_CLASSES = 16;   // class = 15 - min(15, floor(log2(degree + 1)))
constexpr int RM_TILE = 1024;    // vertices per tile of the stable partition

struct RemapDesc {
    const long long* off;
    const int* col;
    const int* w;
    unsigned* tcol;  // [m] key position of each edge's target, rows ordered by class
    int* tw;         // [m] the edge weights in that order
    unsigned* pos;   // [n]
    unsigned* orig;  // [n]
    unsigned char* cls;  // [n] class of each vertex
    int* hist;       // [tiles * RM_CLASSES]: class counts, then their bases
    int n;
    int tiles;
    long long m;
    int tile_begin;  // tiles of earlier remapped graphs
    int pad;
};

__device__ __forceinline__ int rm_class(const long long* off, int v) {
    const unsigned long long d = (unsigned long long)(off[v + 1] - off[v]);
    const int lg = 63 - __clzll(d + 1ull);
    return RM_CLASSES - 1 - (lg < RM_CLASSES - 1 ? lg : RM_CLASSES - 1);
}

// the remapped graph and tile of global tile index g
__device__ __forceinline__ int rm_find(const RemapDesc* R, int nr, int g) {
    int r = 0;
    while (r + 1 < nr && R[r + 1].tile_begin <= g) ++r;
    return r;
}

// class counts of every tile (one wave per tile)
__global__ void k_rm_hist(const RemapDesc* R, int nr, int total_tiles) {
    const int lane = bq::lane_id();
    for (int g = blockIdx.x; g < total_tiles; g += gridDim.x) {
        const RemapDesc& d = R[rm_find(R, nr, g)];
        const int tile = g - d.tile_begin;
        int cnt[RM_CLASSES];
        for (int c = 0; c < RM_CLASSES; ++c) cnt[c] = 0;
        for (int v0 = tile * RM_TILE; v0 < (tile + 1) * RM_TILE && v0 < d.n; v0 += 64) {
            const int v = v0 + lane;
            const int c = v < d.n ? rm_class(d.off, v) : -1;
            for (int k = 0; k < RM_CLASSES; ++k) cnt[k] += __popcll(bq::ballot(c == k));
        }
        if (lane < RM_CLASSES) {
            int x = 0;
            for (int k = 0; k < RM_CLASSES; ++k) x = lane == k ? cnt[k] : x;
            d.hist[tile * RM_CLASSES + lane] = x;
        }
    }
}

// exclusive scan of the counts in (class, tile) order: one workgroup of 1024
// threads per remapped graph
__global__ __launch_bounds__(1024) void k_rm_scan(const RemapDesc* R, int nr) {
    __shared__ int part[1024 / 64];
    for (int r = blockIdx.x; r < nr; r += gridDim.x) {
        const RemapDesc& d = R[r];
        int carry = 0;
        for (int c = 0; c < RM_CLASSES; ++c) {
            for (int t0 = 0; t0 < d.tiles; t0 += 1024) {
                const int t = t0 + (int)threadIdx.x;
                const int x = t < d.tiles ? d.hist[t * RM_CLASSES + c] : 0;
                const int incl = bq::wave_incl_scan(x);
                if (bq::lane_id() == 63) part[threadIdx.x >> 6] = incl;
                __syncthreads();
                int before = carry;
                for (int k = 0; k < (int)(threadIdx.x >> 6); ++k) before += part[k];
                int tot = 0;
                for (int k = 0; k < 1024 / 64; ++k) tot += part[k];
                __syncthreads();
                if (t < d.tiles) d.hist[t * RM_CLASSES + c] = before + incl - x;
                carry += tot;
            }
        }
    }
}

// key position of every vertex: its class's base in its tile plus its rank
// among the tile's vertices of that class (one wave per tile, so positions
// follow vertex ids within a class)
__global__ void k_rm_place(const RemapDesc* R, int nr, int total_tiles) {
    const int lane = bq::lane_id();
    for (int g = blockIdx.x; g < total_tiles; g += gridDim.x) {
        const RemapDesc& d = R[rm_find(R, nr, g)];
        const int tile = g - d.tile_begin;
        int next = lane < RM_CLASSES ? d.hist[tile * RM_CLASSES + lane] : 0;
        for (int v0 = tile * RM_TILE; v0 < (tile + 1) * RM_TILE && v0 < d.n; v0 += 64) {
            const int v = v0 + lane;
            const int c = v < d.n ? rm_class(d.off, v) : -1;
            unsigned p = 0;
            for (int k = 0; k < RM_CLASSES; ++k) {
                const unsigned long long mk = bq::ballot(c == k);
                const int base = __shfl(next, k, 64);
                if (c == k) p = (unsigned)(base + bq::rank_in(mk));
                if (lane == k) next += __popcll(mk);
            }
            if (v < d.n) {
                d.pos[v] = p;
                d.orig[p] = (unsigned)v;
                d.cls[v] = (unsigned char)c;
            }
        }
    }
}

// Every row of every remapped graph, reordered by the class of its targets
// (stable, so each class keeps the row's order), into tcol (target key
// positions) and tw (weights): a wave's lanes then read the keys of the
// most pointed-at targets first and side by side. One wave per row.
__global__ void k_rm_rows(const RemapDesc* R, int nr) {
    const int lane = bq::lane_id();
    const long long waves = (long long)gridDim.x * (blockDim.x >> 6);
    const long long wave = (long long)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    for (int r = 0; r < nr; ++r) {
        const RemapDesc& d = R[r];
        for (long long u = wave; u < d.n; u += waves) {
            const long long s = d.off[u], e = d.off[u + 1];
            int cnt[RM_CLASSES];
            for (int k = 0; k < RM_CLASSES; ++k) cnt[k] = 0;
            for (long long e0 = s; e0 < e; e0 += 64) {
                const long long i = e0 + lane;
                const int c = i < e ? (int)d.cls[d.col[i]] : -1;
                for (int k = 0; k < RM_CLASSES; ++k) cnt[k] += __popcll(bq::ballot(c == k));
            }
            int base[RM_CLASSES];
            int run = 0;
            for (int k = 0; k < RM_CLASSES; ++k) {
                base[k] = run;
                run += cnt[k];
            }
            for (long long e0 = s; e0 < e; e0 += 64) {
                const long long i = e0 + lane;
                const bool live = i < e;
                const int v = live ? d.col[i] : 0;
                const int c = live ? (int)d.cls[v] : -1;
                long long at = 0;
                for (int k = 0; k < RM_CLASSES; ++k) {
                    const unsigned long long mk = bq::ballot(c == k);
                    if (c == k) at = s + base[k] + bq::rank_in(mk);
                    base[k] += __popcll(mk);
                }
                if (live) {
                    d.tcol[at] = d.pos[v];
                    d.tw[at] = d.w[i];
                }
            }
        }
    }
}

// Workgroups are dispatched to the XCDs in turn (workgroup i on XCD i mod 8),
// so workgroup i claims from list i mod n_lists.
constexpr int NLIST = 8;

struct BatchCtl {
    bq::Word cursor[NLIST];  // next entry of each claim list
    bq::Word stats[bq::ST_N];
};

__global__ __launch_bounds__(BINIT_WG) void k_binit(const InstDesc* D, const Unit* units,
                                                    int n_units, int* partials, BatchCtl* bc,
                                                    unsigned long long* reached) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        for (int x = 0; x < NLIST; ++x) bc->cursor[x].v = 0ull;
        for (int i = 0; i < bq::ST_N; ++i) bc->stats[i].v = 0ull;
    }
    __shared__ int slo[BINIT_WG / 64], shi[BINIT_WG / 64];
    for (int u = blockIdx.x; u < n_units; u += gridDim.x) {
        const Unit un = units[u];
        const InstDesc& d = D[un.inst];
        const SolveArgs& a = d.a;
        const long long srckey = pack_key(0, (1u << (a.shift - 1u)) - 1u, a.shift);
        const long long spos = (long long)pos_of(a, (unsigned)a.src);
        for (long long v = un.v0 + threadIdx.x; v < un.v1; v += blockDim.x)
            a.key[v] = (v == spos) ? srckey : KEY_INF;
        int lo = INT_MAX, hi = INT_MIN;
        for (long long e = un.e0 + threadIdx.x; e < un.e1; e += blockDim.x) {
            const int x = a.w[e];
            lo = x < lo ? x : lo;
            hi = x > hi ? x : hi;
        }
        for (int off = 32; off > 0; off >>= 1) {
            const int x = __shfl_xor(lo, off, 64), y = __shfl_xor(hi, off, 64);
            lo = x < lo ? x : lo;
            hi = y > hi ? y : hi;
        }
        if (bq::lane_id() == 0) {
            slo[threadIdx.x >> 6] = lo;
            shi[threadIdx.x >> 6] = hi;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            for (int i = 1; i < BINIT_WG / 64; ++i) {
                lo = slo[i] < lo ? slo[i] : lo;
                hi = shi[i] > hi ? shi[i] : hi;
            }
            partials[2 * u] = lo;
            partials[2 * u + 1] = hi;
            if (u == d.unit_begin) {
                reached[d.orig] = 0ull;
                bq::Ctrl* c = a.q.ctrl;
                c->pending.v = 1ull;
                c->abort.v = 0ull;
                c->error.v = 0ull;
                c->negcycle.v = 0ull;
                c->aux[0].v = (unsigned long long)(d.unit_end - d.unit_begin);
                for (unsigned sg = 0; sg < a.nq; ++sg)  // dequeue positions at start
                    c[sg].aux[2].v = c[sg].head.v;
                c->aux[1].v = (unsigned long long)LLONG_MIN;  // near / far threshold
                c->busy.v = 0ull;
                c->aux[4].v = bq::now_ticks();
                c->aux[5].v = 0ull;  // finished flag
                for (int i = 0; i < bq::ST_N; ++i) c->stats[i].v = 0ull;
                const unsigned long long pos = c->tail.v;
                const unsigned slot = (unsigned)(pos & (a.q.N - 1ull));
                const unsigned round = (unsigned)(pos >> a.q.logN);
                a.q.slots[slot] = bq::slot_word(2u * round + 1u, (unsigned)spos);
                c->tail.v = pos + 1ull;
                c->count.v = 1ull;
            }
        }
        __syncthreads();
    }
}

template <int B>
// D is read-only for the whole launch (__restrict__): its uniform loads then
// go through the scalar cache, and the descriptor of the query a workgroup
// works on stays in scalar registers instead of taking vector ones.
// claim: NLIST + 1 list offsets, then the entries (descriptor indices) of
// list x at [claim[x], claim[x + 1]) after that header.
__global__ __launch_bounds__(SOLVE_WG, SSSP_MIN_WAVES) void k_bsolve(const InstDesc* __restrict__ D, int count,
                                                     const int* claim, int n_lists,
                                                     BatchCtl* bc) {
    __shared__ WaveLds<B, false> lds[WAVES_PER_WG];
    __shared__ WgShared S;
    __shared__ int s_inst;
    WaveLds<B, false>& L = lds[threadIdx.x >> 6];
    const int wid = (int)(threadIdx.x >> 6);
    WaveStats st{};
    int help = (int)(blockIdx.x % (unsigned)count);
    const int x = (int)(blockIdx.x % (unsigned)n_lists);
    const int* list = claim + NLIST + 1;
    const int lo = claim[x], hi = claim[x + 1];
    bool own = true;
    for (;;) {
        if (threadIdx.x == 0) {
            int i = -1;
            if (own) {
                const unsigned long long c = bq::add_rlx(&bc->cursor[x].v, 1ull);
                if (c < (unsigned long long)(hi - lo)) i = list[lo + (int)c];
                else own = false;
            }
            if (i < 0 && hi > lo) {
                // an unfinished query of this list first (its keys are in
                // this XCD's L2), starting at a place of its own
                const int len = hi - lo;
                const int s0 = (int)((blockIdx.x / (unsigned)n_lists) % (unsigned)len);
                for (int k = 0; k < len; ++k) {
                    const int e = lo + (s0 + k) % len;
                    const int j = list[e];
                    if (k > 0 && e > lo && list[e - 1] == j) continue;  // same query again
                    if (bq::ld_rlx(&D[j].a.q.ctrl->aux[5].v) == 0ull) {
                        i = j;
                        break;
                    }
                }
            }
            if (i < 0) {
                for (int k = 0; k < count; ++k) {
                    const int j = (help + k) % count;
                    if (bq::ld_rlx(&D[j].a.q.ctrl->aux[5].v) == 0ull) {
                        i = j;
                        break;
                    }
                }
                if (i >= 0) help = (i + 1) % count;
            }
            s_inst = i;
            S.poller = -1;
            S.wake = 0u;
            S.done = 0;
        }
        __syncthreads();
        const int i = __builtin_amdgcn_readfirstlane(s_inst);  // workgroup-uniform
        if (i < 0) break;
        const SolveArgs a = D[i].a;
        solve_instance<B>(a, L, S, wid, st);
        __syncthreads();
        if (threadIdx.x == 0) bq::st_rlx(&a.q.ctrl->aux[5].v, 1ull);
        __syncthreads();
    }
    flush_stats(bc->stats, st);
}

// Unpack, and count the query's reached edges (out-degrees of reached
// vertices) for throughput figures.
__global__ void k_bunpack(const InstDesc* D, const Unit* units, int n_units,
                          long long* results, unsigned long long* reached_edges) {
    for (int u = blockIdx.x; u < n_units; u += gridDim.x) {
        const Unit un = units[u];
        const InstDesc& d = D[un.inst];
        const SolveArgs& a = d.a;
        const long long dmax = KEY_INF >> a.shift;
        const unsigned pmask = (1u << (a.shift - 1u)) - 1u;
        unsigned long long redges = 0;
        for (long long v = un.v0 + threadIdx.x; v < un.v1; v += blockDim.x) {
            const long long k = a.key[pos_of(a, (unsigned)v)];
            if (is_neg_key(k)) {  // minus infinity (marking mode)
                d.dist[v] = LLONG_MIN;
                redges += (unsigned long long)(a.off[v + 1] - a.off[v]);
                if (d.pred) d.pred[v] = -1;
                continue;
            }
            const long long dd = k >> a.shift;
            const bool reached = dd != dmax;
            d.dist[v] = reached ? dd : LLONG_MAX;
            if (reached) redges += (unsigned long long)(a.off[v + 1] - a.off[v]);
            if (d.pred)
                d.pred[v] = (reached && v != a.src)
                                ? (int)(((unsigned long long)k >> 1) & pmask)
                                : -1;
        }
        for (int off = 32; off > 0; off >>= 1) redges += __shfl_xor(redges, off, 64);
        if (bq::lane_id() == 0 && redges) bq::add_rlx(&reached_edges[d.orig], redges);
        if (u == d.unit_begin && threadIdx.x == 0) {
            const bq::Ctrl* c = a.q.ctrl;
            results[d.orig] = (long long)(c->negcycle.v & 1ull) |
                              ((long long)c->error.v << 8) | ((long long)c->abort.v << 16);
        }
    }
}

unsigned bkey_shift(int n) {
    unsigned pb = 0;
    while ((1ull << pb) < (unsigned long long)n + 1ull) ++pb;
    return pb + 1u;
}

unsigned long long pow2ceil(unsigned long long x) {
    unsigned long long p = 1ull;
    while (p < x) p <<= 1;
    return p;
}

}  // namespace

struct sssp_batch {
    int device;
    int max_inst;
    long long max_n, max_m;
    size_t slot_cap, chunk_cap, max_units, max_claim;
    unsigned long long* slots;
    unsigned* chunks;
    bq::Ctrl* ctrls;
    // degree-class key layouts of shared graphs: keys of the queries on
    // them, remapped targets, positions, original ids, per-tile class counts
    long long* keys;
    unsigned* rm_tcol;
    int* rm_tw;
    unsigned char* rm_cls;
    unsigned* rm_pos;
    unsigned* rm_orig;
    int* rm_hist;
    size_t key_cap, rm_cap_m, rm_cap_n, rm_cap_tiles;
    RemapDesc* d_rm;
    RemapDesc* h_rm;
    InstDesc* d_desc;
    Unit* d_units;
    int* d_claim;
    int* d_partials;
    long long* d_results;
    unsigned long long* d_reached;
    BatchCtl* d_bc;
    InstDesc* h_desc;
    Unit* h_units;
    int* h_claim;
    long long* h_results;
    unsigned long long* h_reached;
    BatchCtl* h_bc;
    int started;  // queries of a started, not yet finished call (0 = none)
    hipStream_t stream;
    hipEvent_t ev0, ev1, ev_in, ev_done;
    std::vector<unsigned long long> layout;
    bool dirty;
    // autotuned launches by shape bucket (sssp_batch_autotune)
    std::map<unsigned long long, std::pair<bq_launch, double>> tuned;
    hipGraphExec_t exec;
    hipGraph_t graph;
    unsigned long long graph_key[8];
    int per_cu[3];
    sssp_stats last;
};

namespace {

bq_status batch_launch_kernels(sssp_batch* b, int count, int n_units, int n_lists, int grid,
                               int B, int nr, int rm_tiles) {
    hipStream_t s = b->stream;
    const int ug = n_units < 2048 ? n_units : 2048;
    if (nr > 0) {
        const int tg = rm_tiles < 4096 ? rm_tiles : 4096;
        hipLaunchKernelGGL(k_rm_hist, dim3(tg), dim3(64), 0, s, b->d_rm, nr, rm_tiles);
        hipLaunchKernelGGL(k_rm_scan, dim3(nr), dim3(1024), 0, s, b->d_rm, nr);
        hipLaunchKernelGGL(k_rm_place, dim3(tg), dim3(64), 0, s, b->d_rm, nr, rm_tiles);
        hipLaunchKernelGGL(k_rm_rows, dim3(2048), dim3(256), 0, s, b->d_rm, nr);
    }
    hipLaunchKernelGGL(k_binit, dim3(ug), dim3(BINIT_WG), 0, s, b->d_desc, b->d_units, n_units,
                       b->d_partials, b->d_bc, b->d_reached);
    switch (B) {
        case 64:
            hipLaunchKernelGGL(k_bsolve<64>, dim3(grid), dim3(SOLVE_WG), 0, s, b->d_desc, count,
                               b->d_claim, n_lists, b->d_bc);
            break;
        case 128:
            hipLaunchKernelGGL(k_bsolve<128>, dim3(grid), dim3(SOLVE_WG), 0, s, b->d_desc, count,
                               b->d_claim, n_lists, b->d_bc);
            break;
        default:
            hipLaunchKernelGGL(k_bsolve<256>, dim3(grid), dim3(SOLVE_WG), 0, s, b->d_desc, count,
                               b->d_claim, n_lists, b->d_bc);
            break;
    }
    hipLaunchKernelGGL(k_bunpack, dim3(ug), dim3(256), 0, s, b->d_desc, b->d_units, n_units,
                       b->d_results, b->d_reached);
    BQ_HIP_TRY(hipGetLastError());
    return BQ_OK;
}

int batch_max_grid(sssp_batch* b, int B) {
    const int slot = B == 64 ? 0 : (B == 128 ? 1 : 2);
    int& pc = b->per_cu[slot];
    if (pc == 0) {
        hipError_t e;
        if (B == 64)
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&pc, k_bsolve<64>, SOLVE_WG, 0);
        else if (B == 128)
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&pc, k_bsolve<128>, SOLVE_WG, 0);
        else
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&pc, k_bsolve<256>, SOLVE_WG, 0);
        if (e != hipSuccess || pc < 1) pc = 1;
    }
    return pc * bqh::device_cus();
}

}  // namespace

extern "C" {

bq_status sssp_batch_create(int32_t max_instances, int64_t max_total_n, int64_t max_total_m,
                            sssp_batch** out) {
    if (!out || max_instances < 1 || max_total_n < 1 || max_total_m < 0) return BQ_EINVAL;
    *out = nullptr;
    sssp_batch* b = new sssp_batch();
    BQ_HIP_TRY(hipGetDevice(&b->device));
    b->max_inst = max_instances;
    b->max_n = max_total_n;
    b->max_m = max_total_m;
    // per query: capacity pow2(scale * (n + m/C + 1)) with scale <= 2 and
    // C >= 64, at least 4096 -> at most 4 * (n + m/64 + 1) + 4096 each
    b->slot_cap = 3 * ((size_t)(4 * (max_total_n + max_total_m / 64 + max_instances)) +
                       (size_t)max_instances * 4096);  // vertex queue, chunk lane, far queue
    b->chunk_cap = (size_t)(max_total_m / 64 + max_instances);
    b->max_units = (size_t)((max_total_n + max_total_m) / UNIT + 2 * max_instances);
    b->max_claim = (size_t)(8 * 4096 + max_instances + NLIST + 1);
    // a remapped graph is shared by two or more queries, so the remapped
    // graphs hold at most half of the vertices and edges of a batch
    b->key_cap = (size_t)max_total_n;
    b->rm_cap_n = (size_t)(max_total_n / 2 + 1);
    b->rm_cap_m = (size_t)(max_total_m / 2 + 1);
    b->rm_cap_tiles = b->rm_cap_n / RM_TILE + (size_t)max_instances / 2 + 1;
    if (hipMalloc(&b->slots, sizeof(unsigned long long) * b->slot_cap) != hipSuccess ||
        hipMalloc(&b->keys, sizeof(long long) * b->key_cap) != hipSuccess ||
        hipMalloc(&b->rm_tcol, sizeof(unsigned) * b->rm_cap_m) != hipSuccess ||
        hipMalloc(&b->rm_tw, sizeof(int) * b->rm_cap_m) != hipSuccess ||
        hipMalloc(&b->rm_cls, b->rm_cap_n) != hipSuccess ||
        hipMalloc(&b->rm_pos, sizeof(unsigned) * b->rm_cap_n) != hipSuccess ||
        hipMalloc(&b->rm_orig, sizeof(unsigned) * b->rm_cap_n) != hipSuccess ||
        hipMalloc(&b->rm_hist, sizeof(int) * RM_CLASSES * b->rm_cap_tiles) != hipSuccess ||
        hipMalloc(&b->d_rm, sizeof(RemapDesc) * max_instances) != hipSuccess ||
        hipHostMalloc(&b->h_rm, sizeof(RemapDesc) * max_instances, hipHostMallocDefault) !=
            hipSuccess ||
        hipMalloc(&b->chunks, sizeof(unsigned) * b->chunk_cap) != hipSuccess ||
        hipMalloc(&b->ctrls, sizeof(bq::Ctrl) * max_instances * MAX_Q) != hipSuccess ||
        hipMalloc(&b->d_desc, sizeof(InstDesc) * max_instances) != hipSuccess ||
        hipMalloc(&b->d_units, sizeof(Unit) * b->max_units) != hipSuccess ||
        hipMalloc(&b->d_claim, sizeof(int) * b->max_claim) != hipSuccess ||
        hipMalloc(&b->d_partials, sizeof(int) * 2 * b->max_units) != hipSuccess ||
        hipMalloc(&b->d_results, sizeof(long long) * max_instances) != hipSuccess ||
        hipMalloc(&b->d_reached, sizeof(unsigned long long) * max_instances) != hipSuccess ||
        hipMalloc(&b->d_bc, sizeof(BatchCtl)) != hipSuccess ||
        hipHostMalloc(&b->h_desc, sizeof(InstDesc) * max_instances, hipHostMallocDefault) !=
            hipSuccess ||
        hipHostMalloc(&b->h_units, sizeof(Unit) * b->max_units, hipHostMallocDefault) !=
            hipSuccess ||
        hipHostMalloc(&b->h_claim, sizeof(int) * b->max_claim, hipHostMallocDefault) !=
            hipSuccess ||
        hipHostMalloc(&b->h_results, sizeof(long long) * max_instances, hipHostMallocDefault) !=
            hipSuccess ||
        hipHostMalloc(&b->h_reached, sizeof(unsigned long long) * max_instances,
                      hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc(&b->h_bc, sizeof(BatchCtl), hipHostMallocDefault) != hipSuccess) {
        sssp_batch_destroy(b);
        return BQ_ENOMEM;
    }
    BQ_HIP_TRY(hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking));
    BQ_HIP_TRY(hipEventCreate(&b->ev0));
    BQ_HIP_TRY(hipEventCreate(&b->ev1));
    BQ_HIP_TRY(hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming));
    BQ_HIP_TRY(hipEventCreateWithFlags(&b->ev_done, hipEventDisableTiming));
    b->dirty = true;
    BQ_HIP_TRY(hipMemsetAsync(b->slots, 0, sizeof(unsigned long long) * b->slot_cap, b->stream));
    BQ_HIP_TRY(hipMemsetAsync(b->ctrls, 0, sizeof(bq::Ctrl) * max_instances * MAX_Q,
                              b->stream));
    BQ_HIP_TRY(hipStreamSynchronize(b->stream));
    b->dirty = false;
    *out = b;
    return BQ_OK;
}

bq_status sssp_batch_destroy(sssp_batch* b) {
    if (!b) return BQ_OK;
    (void)hipDeviceSynchronize();
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->slots) (void)hipFree(b->slots);
    if (b->chunks) (void)hipFree(b->chunks);
    if (b->keys) (void)hipFree(b->keys);
    if (b->rm_tcol) (void)hipFree(b->rm_tcol);
    if (b->rm_tw) (void)hipFree(b->rm_tw);
    if (b->rm_cls) (void)hipFree(b->rm_cls);
    if (b->rm_pos) (void)hipFree(b->rm_pos);
    if (b->rm_orig) (void)hipFree(b->rm_orig);
    if (b->rm_hist) (void)hipFree(b->rm_hist);
    if (b->d_rm) (void)hipFree(b->d_rm);
    if (b->h_rm) (void)hipHostFree(b->h_rm);
    if (b->ctrls) (void)hipFree(b->ctrls);
    if (b->d_desc) (void)hipFree(b->d_desc);
    if (b->d_units) (void)hipFree(b->d_units);
    if (b->d_claim) (void)hipFree(b->d_claim);
    if (b->d_partials) (void)hipFree(b->d_partials);
    if (b->d_results) (void)hipFree(b->d_results);
    if (b->d_reached) (void)hipFree(b->d_reached);
    if (b->d_bc) (void)hipFree(b->d_bc);
    if (b->h_desc) (void)hipHostFree(b->h_desc);
    if (b->h_units) (void)hipHostFree(b->h_units);
    if (b->h_claim) (void)hipHostFree(b->h_claim);
    if (b->h_results) (void)hipHostFree(b->h_results);
    if (b->h_reached) (void)hipHostFree(b->h_reached);
    if (b->h_bc) (void)hipHostFree(b->h_bc);
    if (b->stream) (void)hipStreamDestroy(b->stream);
    if (b->ev0) (void)hipEventDestroy(b->ev0);
    if (b->ev1) (void)hipEventDestroy(b->ev1);
    if (b->ev_in) (void)hipEventDestroy(b->ev_in);
    if (b->ev_done) (void)hipEventDestroy(b->ev_done);
    delete b;
    return BQ_OK;
}

bq_status sssp_batch_last_stats(const sssp_batch* b, sssp_stats* out) {
    if (!b || !out) return BQ_EINVAL;
    *out = b->last;
    return BQ_OK;
}

bq_status sssp_bf_batched_start(sssp_batch* b, int32_t count, const sssp_instance* h_inst,
                                const bq_launch* launch, void* stream) {
    if (!b || !h_inst || count < 1) return BQ_EINVAL;
    if (b->started) return BQ_EBUSY;
    if (count > b->max_inst) return BQ_EBUSY;
    bqh::Launch L = bqh::resolve(launch, 0);
    if (L.batch != 1 && L.batch != 2 && L.batch != 4) return BQ_EINVAL;
    const int B = 64 * L.batch;
    unsigned clog = BDEFAULT_CHUNK_LOG;
    if (L.row_chunk > 0) {
        if (L.row_chunk & (L.row_chunk - 1)) return BQ_EINVAL;
        clog = bqh::log2_exact((unsigned long long)L.row_chunk);
        if (clog < BMIN_CHUNK_LOG || clog > BMAX_CHUNK_LOG) return BQ_EINVAL;
    }
    const int scale = (launch && launch->queue_scale > 0) ? launch->queue_scale : 2;
    if (scale > 2) return BQ_EINVAL;
    if (L.bucket_width < 0) return BQ_EINVAL;
    // queues per segment: vertex queue and chunk lane, plus a far queue with buckets
    const unsigned qps = L.bucket_width > 0 ? 3u : 2u;
    // validate and order by work, biggest first
    long long tot_n = 0, tot_m = 0;
    std::vector<int> order(count);
    for (int i = 0; i < count; ++i) {
        const sssp_instance& x = h_inst[i];
        if (x.n < 1 || x.m < 0 || x.src < 0 || x.src >= x.n || !x.offsets || !x.dist)
            return BQ_EINVAL;
        if (x.m > 0 && (!x.cols || !x.w)) return BQ_EINVAL;
        if ((unsigned long long)x.n + ((unsigned long long)x.m >> clog) + 1ull >= 0xFFFFFFFFull)
            return BQ_EINVAL;
        tot_n += x.n;
        tot_m += x.m;
        order[i] = i;
    }
    if (tot_n > b->max_n || tot_m > b->max_m) return BQ_EBUSY;
    std::vector<long long> work(count);
    for (int i = 0; i < count; ++i) work[i] = h_inst[i].m + h_inst[i].n;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return work[x] > work[y]; });

    const int max_grid = batch_max_grid(b, B);
    // default: about one workgroup per 16K units of n + m/16 of each query
    // (the single-query solver's rule), at least one per query; more waves
    // than the work can feed only raise the relaxations per edge
    long long want = 0;
    for (int i = 0; i < count; ++i) {
        const long long units = (long long)h_inst[i].n + h_inst[i].m / 16;
        want += units / 16384 > 1 ? units / 16384 : 1;
    }
    int grid = L.wg_count > 0 ? L.wg_count : (want < max_grid ? (int)want : max_grid);
    if (grid > max_grid) grid = max_grid;

    // layout: queue slots, chunk tables, units, claim list
    std::vector<unsigned long long> layout;
    layout.reserve(3 * count + 2);
    size_t slot_off = 0, chunk_off = 0;
    int n_units = 0, n_claim = 0;
    std::vector<std::vector<int>> lists(NLIST);
    std::vector<long long> list_work(NLIST, 0);
    long long tot_work = 0;
    for (int i = 0; i < count; ++i) tot_work += work[i];
    // workgroups per query in proportion to its share of the work (at least
    // one); a query whose share fits one XCD's workgroups is confined to one
    // claim list, a bigger one is spread over all lists
    const int n_lists = grid < NLIST ? grid : NLIST;
    std::vector<long long> tgts(count);
    std::vector<char> confined(count);
    for (int k = 0; k < count; ++k) {
        long long tgt = tot_work > 0 ? (long long)grid * work[order[k]] / tot_work : 1;
        if (tgt < 1) tgt = 1;
        tgts[k] = tgt;
        confined[k] = n_lists > 1 && tgt * n_lists <= grid;
    }
    // queue capacity of each query, and its segments: a query that can feed
    // 16 or more workgroups and is spread over the XCDs gets up to MAX_SEG
    // queue segments (one per XCD, as in the single-query solver) while the
    // slot arena has room left over after every query's first segment,
    // biggest queries first; a confined query keeps one (its workgroups all
    // have the same home)
    std::vector<unsigned long long> caps(count);
    std::vector<unsigned> nsegs(count, 1u);
    {
        unsigned long long base = 0;
        for (int k = 0; k < count; ++k) {
            const sssp_instance& x = h_inst[order[k]];
            const unsigned long long need =
                (unsigned long long)x.n + ((unsigned long long)x.m >> clog) + 1ull;
            unsigned long long cap = pow2ceil((unsigned long long)scale * need);
            if (cap < 4096ull) cap = 4096ull;
            caps[k] = cap;
            base += qps * cap;
        }
        unsigned long long spare = base < b->slot_cap ? b->slot_cap - base : 0ull;
        for (int k = 0; k < count; ++k) {
            const sssp_instance& x = h_inst[order[k]];
            const long long units = (long long)x.n + x.m / 16;
            if (units / 16384 < 16 || confined[k]) continue;
            unsigned long long extra = spare / (qps * caps[k]);
            if (extra > MAX_SEG - 1) extra = MAX_SEG - 1;
            nsegs[k] = 1u + (unsigned)extra;
            spare -= qps * extra * caps[k];
        }
    }
    // Graphs that two or more queries share get the degree-class key layout:
    // their queries keep keys in the workspace at key positions ordered by
    // out-degree class, highest first, then by vertex id, so that the keys
    // most edges point at pack into few cache lines. Queries on a graph of
    // their own keep their keys in their dist buffers.
    std::vector<int> rm_of(count, -1);
    int nr = 0, rm_tiles = 0;
    {
        size_t rm_m = 0, rm_n = 0, key_need = 0;
        std::map<std::tuple<const void*, const void*, const void*, int, long long>,
                 std::vector<int>> shared;
        if (!(L.flags & BQ_F_NOREMAP))
            for (int k = 0; k < count; ++k) {
                const sssp_instance& x = h_inst[order[k]];
                shared[std::make_tuple((const void*)x.offsets, (const void*)x.cols,
                                       (const void*)x.w, x.n, (long long)x.m)]
                    .push_back(k);
            }
        for (auto& kv : shared) {
            const std::vector<int>& ks = kv.second;
            if (ks.size() < 2) continue;
            const sssp_instance& x = h_inst[order[ks[0]]];
            const int tiles = (x.n + RM_TILE - 1) / RM_TILE;
            if (rm_m + (size_t)x.m > b->rm_cap_m || rm_n + (size_t)x.n > b->rm_cap_n ||
                (size_t)(rm_tiles + tiles) > b->rm_cap_tiles ||
                key_need + (size_t)x.n * ks.size() > b->key_cap)
                continue;
            RemapDesc& R = b->h_rm[nr];
            R.off = (const long long*)x.offsets;
            R.col = (const int*)x.cols;
            R.w = (const int*)x.w;
            R.tcol = b->rm_tcol + rm_m;
            R.tw = b->rm_tw + rm_m;
            R.cls = b->rm_cls + rm_n;
            R.pos = b->rm_pos + rm_n;
            R.orig = b->rm_orig + rm_n;
            R.hist = b->rm_hist + (size_t)rm_tiles * RM_CLASSES;
            R.n = x.n;
            R.tiles = tiles;
            R.m = (long long)x.m;
            R.tile_begin = rm_tiles;
            R.pad = 0;
            rm_m += (size_t)x.m;
            rm_n += (size_t)x.n;
            rm_tiles += tiles;
            key_need += (size_t)x.n * ks.size();
            for (int k : ks) rm_of[k] = nr;
            ++nr;
        }
    }
    size_t key_off = 0;
    for (int k = 0; k < count; ++k) {
        const int i = order[k];
        const sssp_instance& x = h_inst[i];
        const unsigned long long cap = caps[k];
        const unsigned nseg = nsegs[k];
        const size_t chunks = (size_t)((unsigned long long)x.m >> clog) + 1;
        const long long big = x.n > x.m ? x.n : x.m;
        const int ku = (int)((big + UNIT - 1) / UNIT);
        if (slot_off + qps * nseg * cap > b->slot_cap || chunk_off + chunks > b->chunk_cap ||
            (size_t)(n_units + ku) > b->max_units)
            return BQ_EBUSY;
        InstDesc& d = b->h_desc[k];
        memset(&d, 0, sizeof d);
        SolveArgs& a = d.a;
        a.q.slots = (decltype(a.q.slots))(b->slots + slot_off);
        a.q.ctrl = (decltype(a.q.ctrl))(b->ctrls + (size_t)k * MAX_Q);
        a.q.sig = (decltype(a.q.sig))a.q.ctrl;
        a.q.logN = bqh::log2_exact(cap);
        a.q.pad = 0;
        a.q.N = cap;
        a.off = (decltype(a.off))x.offsets;
        a.col = (decltype(a.col))x.cols;
        a.w = (decltype(a.w))x.w;
        if (rm_of[k] >= 0) {
            const RemapDesc& R = b->h_rm[rm_of[k]];
            a.key = (decltype(a.key))(b->keys + key_off);
            key_off += (size_t)x.n;
            a.tcol = (decltype(a.tcol))R.tcol;
            a.tw = (decltype(a.tw))R.tw;
            a.orig = (decltype(a.orig))R.orig;
            a.pos = (decltype(a.pos))R.pos;
        } else {
            a.key = (decltype(a.key))x.dist;
            a.tcol = nullptr;
            a.tw = nullptr;
            a.orig = nullptr;
            a.pos = nullptr;
        }
        a.chunk_owner = (decltype(a.chunk_owner))(b->chunks + chunk_off);
        a.wrange = (decltype(a.wrange))(b->d_partials + 2 * n_units);
        a.n = x.n;
        a.src = x.src;
        a.m = (long long)x.m;
        a.shift = bkey_shift(x.n);
        a.chunk_log = clog;
        a.limit = L.limit;
        a.deadline = 10ull * L.limit;
        a.trace = nullptr;
        a.trace_shift = 0;
        a.trace_cap = 0;
        a.bwd = (L.flags & BQ_F_BWD) ? 1u : 0u;
        a.nseg = nseg;
        a.nq = qps * nseg;
        a.bucket_width = L.bucket_width;
        a.neginf = (L.flags & BQ_F_NEGINF) ? 1u : 0u;
        a.fan_bulk = 1u;
        d.dist = (long long*)x.dist;
        d.pred = (int*)x.pred;
        d.orig = i;
        d.unit_begin = n_units;
        for (int j = 0; j < ku; ++j) {
            Unit& un = b->h_units[n_units + j];
            un.inst = k;
            un.pad = 0;
            un.v0 = (long long)x.n * j / ku;
            un.v1 = (long long)x.n * (j + 1) / ku;
            un.e0 = (long long)x.m * j / ku;
            un.e1 = (long long)x.m * (j + 1) / ku;
        }
        n_units += ku;
        d.unit_end = n_units;
        // claim entries: biggest queries first (spread ones round the
        // lists), each confined query on the list with the least work so far
        if (confined[k]) {
            int best = 0;
            for (int l = 1; l < n_lists; ++l)
                if (list_work[l] < list_work[best]) best = l;
            for (long long t = 0; t < tgts[k]; ++t) lists[best].push_back(k);
            list_work[best] += work[i];
        } else {
            for (long long t = 0; t < tgts[k]; ++t) {
                const int l = (int)(t % n_lists);
                lists[l].push_back(k);
                list_work[l] += work[i] / tgts[k];
            }
        }
        layout.push_back(cap);
        layout.push_back(slot_off);
        layout.push_back(nseg);
        slot_off += qps * nseg * cap;  // vertex queues, chunk lanes (and far queues)
        chunk_off += chunks;
    }
    // the claim array: list offsets, then the lists one after another
    {
        size_t total = NLIST + 1;
        for (const auto& l : lists) total += l.size();
        if (total > b->max_claim) return BQ_EBUSY;
        int pos = 0;
        for (int l = 0; l < NLIST; ++l) {
            b->h_claim[l] = pos;
            for (int e : lists[l]) b->h_claim[NLIST + 1 + pos++] = e;
        }
        b->h_claim[NLIST] = pos;
        n_claim = (int)total;
    }
    hipStream_t cs = bqh::as_stream(stream);
    hipStream_t s = b->stream;
    // queue state is reusable only if every query keeps the same slots and a
    // clean end; otherwise zero the slots and control blocks first
    if (b->dirty || layout != b->layout) {
        BQ_HIP_TRY(hipMemsetAsync(b->slots, 0, sizeof(unsigned long long) * slot_off, s));
        BQ_HIP_TRY(hipMemsetAsync(b->ctrls, 0, sizeof(bq::Ctrl) * count * MAX_Q, s));
        b->layout = layout;
        b->dirty = false;
    }
    BQ_HIP_TRY(hipMemcpyAsync(b->d_desc, b->h_desc, sizeof(InstDesc) * count,
                              hipMemcpyHostToDevice, s));
    BQ_HIP_TRY(hipMemcpyAsync(b->d_units, b->h_units, sizeof(Unit) * n_units,
                              hipMemcpyHostToDevice, s));
    BQ_HIP_TRY(hipMemcpyAsync(b->d_claim, b->h_claim, sizeof(int) * n_claim,
                              hipMemcpyHostToDevice, s));
    if (nr > 0)
        BQ_HIP_TRY(hipMemcpyAsync(b->d_rm, b->h_rm, sizeof(RemapDesc) * nr,
                                  hipMemcpyHostToDevice, s));
    // the caller's stream must be done with the inputs
    BQ_HIP_TRY(hipEventRecord(b->ev_in, cs));
    BQ_HIP_TRY(hipStreamWaitEvent(s, b->ev_in, 0));

    BQ_HIP_TRY(hipEventRecord(b->ev0, s));
    if (L.flags & BQ_F_GRAPH) {
        const unsigned long long key[8] = {(unsigned long long)count, (unsigned long long)n_units,
                                           (unsigned long long)n_claim, (unsigned long long)grid,
                                           (unsigned long long)B, (unsigned long long)n_lists,
                                           (unsigned long long)nr,
                                           (unsigned long long)rm_tiles};
        if (!b->exec || memcmp(key, b->graph_key, sizeof key) != 0) {
            if (b->exec) {
                (void)hipGraphExecDestroy(b->exec);
                b->exec = nullptr;
            }
            if (b->graph) {
                (void)hipGraphDestroy(b->graph);
                b->graph = nullptr;
            }
            BQ_HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
            bq_status st = batch_launch_kernels(b, count, n_units, n_lists, grid, B, nr, rm_tiles);
            hipGraph_t g = nullptr;
            hipError_t ce = hipStreamEndCapture(s, &g);
            if (st != BQ_OK) return st;
            BQ_HIP_TRY(ce);
            b->graph = g;
            BQ_HIP_TRY(hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0));
            memcpy(b->graph_key, key, sizeof key);
        }
        BQ_HIP_TRY(hipGraphLaunch(b->exec, s));
    } else {
        bq_status st = batch_launch_kernels(b, count, n_units, n_lists, grid, B, nr, rm_tiles);
        if (st != BQ_OK) return st;
    }
    BQ_HIP_TRY(hipEventRecord(b->ev1, s));
    BQ_HIP_TRY(hipMemcpyAsync(b->h_results, b->d_results, sizeof(long long) * count,
                              hipMemcpyDeviceToHost, s));
    BQ_HIP_TRY(hipMemcpyAsync(b->h_reached, b->d_reached, sizeof(unsigned long long) * count,
                              hipMemcpyDeviceToHost, s));
    BQ_HIP_TRY(hipMemcpyAsync(b->h_bc, b->d_bc, sizeof(BatchCtl), hipMemcpyDeviceToHost, s));
    BQ_HIP_TRY(hipEventRecord(b->ev_done, s));
    b->started = count;
    b->last.grid = grid;
    return BQ_OK;
}

bq_status sssp_batch_finish(sssp_batch* b, int32_t* h_neg_cycle, int64_t* h_reached_edges,
                            int32_t wait) {
    if (!b || !h_neg_cycle) return BQ_EINVAL;
    const int count = b->started;
    if (count == 0) return BQ_EINVAL;
    if (wait) {
        BQ_HIP_TRY(hipEventSynchronize(b->ev_done));
    } else {
        const hipError_t q = hipEventQuery(b->ev_done);
        if (q == hipErrorNotReady) return BQ_EBUSY;
        BQ_HIP_TRY(q);
    }
    b->started = 0;
    float ms = 0.f;
    BQ_HIP_TRY(hipEventElapsedTime(&ms, b->ev0, b->ev1));
    const BatchCtl* h = b->h_bc;
    const int grid = b->last.grid;
    b->last = sssp_stats{};
    b->last.dequeued = h->stats[bq::ST_DEQ].v;
    b->last.relaxations = h->stats[bq::ST_RELAX].v;
    b->last.pushes = h->stats[bq::ST_PUSH].v;
    b->last.fanout = h->stats[bq::ST_FANOUT].v;
    b->last.batches = h->stats[bq::ST_BATCH].v;
    b->last.walks = h->stats[bq::ST_WALK].v;
    b->last.improvements = h->stats[bq::ST_IMPROVE].v;
    b->last.idle_polls = h->stats[bq::ST_POLL].v;
    b->last.ticket_spins = h->stats[bq::ST_SPIN].v;
    b->last.ms = ms;
    b->last.solve_ms = ms;
    b->last.grid = grid;
    b->last.wg_size = SOLVE_WG;
    bq_status ret = BQ_OK;
    for (int i = 0; i < count; ++i) {
        const long long r = b->h_results[i];
        h_neg_cycle[i] = (int32_t)(r & 1);
        if (h_reached_edges) h_reached_edges[i] = (int64_t)b->h_reached[i];
        const long long err = (r >> 8) & 0xff;
        if (r & ~1ll) b->dirty = true;  // a stopped query leaves its queue non-quiescent
        if (err == bq::ERR_RANGE && ret == BQ_OK) ret = BQ_ERANGE;
        else if (err == bq::ERR_FULL && ret == BQ_OK) ret = BQ_EOVERFLOW;
        else if (err != 0 && ret == BQ_OK) ret = BQ_ETIMEOUT;
    }
    return ret;
}

bq_status sssp_bf_batched(sssp_batch* b, int32_t count, const sssp_instance* h_inst,
                          int32_t* h_neg_cycle, const bq_launch* launch, void* stream) {
    if (!h_neg_cycle) return BQ_EINVAL;
    bq_status st = sssp_bf_batched_start(b, count, h_inst, launch, stream);
    if (st != BQ_OK) return st;
    return sssp_batch_finish(b, h_neg_cycle, nullptr, 1);
}

bq_status sssp_batch_autotune(sssp_batch* b, int32_t count, const sssp_instance* h_inst,
                              const bq_launch* base, int32_t reps, bq_launch* h_best,
                              double* h_best_ms, void* stream) {
    if (!b || !h_inst || !h_best || !h_best_ms || count < 1) return BQ_EINVAL;
    if (reps < 1) reps = 3;
    bq_launch L = {};
    if (base) L = *base;
    // shape bucket: powers of two of the query count and of the total
    // vertices and edges, plus the caller's flags
    unsigned long long tn = 0, tm = 0;
    for (int i = 0; i < count; ++i) {
        tn += (unsigned long long)(h_inst[i].n > 0 ? h_inst[i].n : 0);
        tm += (unsigned long long)(h_inst[i].m > 0 ? h_inst[i].m : 0);
    }
    const unsigned long long bucket = ((unsigned long long)bqh::log2_exact(count) << 48) |
                                      ((unsigned long long)bqh::log2_exact(tn + 1) << 40) |
                                      ((unsigned long long)bqh::log2_exact(tm + 1) << 32) |
                                      (unsigned long long)L.flags;
    auto hit = b->tuned.find(bucket);
    if (hit != b->tuned.end()) {
        *h_best = hit->second.first;
        *h_best_ms = hit->second.second;
        return BQ_OK;
    }
    std::vector<int32_t> neg(count);
    double best = 1e300;
    bq_launch bestL = L;
    // median of the runs, and a 3 % margin before a new shape replaces the
    // fastest so far (the work of asynchronous solves varies run to run)
    auto trial = [&](bq_launch t) -> bq_status {
        std::vector<double> ts;
        for (int r = 0; r < reps; ++r) {
            bq_status st = sssp_bf_batched(b, count, h_inst, neg.data(), &t, stream);
            if (st != BQ_OK) return st;
            ts.push_back(b->last.ms);
        }
        std::sort(ts.begin(), ts.end());
        const double med = (ts[(ts.size() - 1) / 2] + ts[ts.size() / 2]) / 2.0;
        if (med < best * (best < 1e300 ? 0.97 : 1.0)) {
            best = med;
            bestL = t;
        }
        return BQ_OK;
    };
    const int max_grid = batch_max_grid(b, 64);
    for (int wgs = 16; wgs <= max_grid; wgs *= 2) {
        bq_launch t = L;
        t.wg_count = wgs;
        t.ticket_batch = 1;
        bq_status st = trial(t);
        if (st != BQ_OK) return st;
    }
    {
        bq_launch t = L;
        t.wg_count = max_grid;
        t.ticket_batch = 1;
        bq_status st = trial(t);
        if (st != BQ_OK) return st;
    }
    const bq_launch cur = bestL;
    for (int chunk : {256, 4096}) {
        bq_launch t = cur;
        t.row_chunk = chunk;
        bq_status st = trial(t);
        if (st != BQ_OK) return st;
    }
    {
        const bq_launch at = bestL;
        for (int bb : {2, 4}) {
            bq_launch t = at;
            t.ticket_batch = bb;
            bq_status st = trial(t);
            if (st != BQ_OK) return st;
        }
        bq_launch t = bestL;
        t.queue_scale = 1;  // queue capacity pow2(n + m/C + 1) instead of twice that
        bq_status st = trial(t);
        if (st != BQ_OK) return st;
        t = bestL;
        t.flags |= BQ_F_NOREMAP;  // keys of shared graphs in vertex order
        st = trial(t);
        if (st != BQ_OK) return st;
    }
    b->tuned[bucket] = std::make_pair(bestL, best);
    *h_best = bestL;
    *h_best_ms = best;
    return BQ_OK;
}

}  // extern "C"
