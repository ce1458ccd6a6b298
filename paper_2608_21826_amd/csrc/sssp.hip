// Host API of the single-query queue-based Bellman-Ford SSSP (Section III.C):
// context, launch sequence (init, persistent solver, unpack; kernels in
// sssp_kernels.hpp), autotuner.
#include <hip/hip_runtime.h>
#include <limits.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "csr_device.hpp"
#include "host_common.hpp"
#include "sssp_kernels.hpp"


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

constexpr unsigned DEFAULT_CHUNK_LOG = 7;   // rows longer than 128 edges are split
constexpr unsigned MIN_CHUNK_LOG = 6;       // smallest row chunk a launch may ask for
constexpr unsigned MAX_CHUNK_LOG = 16;
constexpr int TRACE_CAP = 4096;

bq_status ctx_reset_queue(sssp_ctx* c, hipStream_t s) {
    BQ_HIP_TRY(hipMemsetAsync(c->slots, 0,
                              sizeof(unsigned long long) * c->capacity * MAX_Q, s));
    BQ_HIP_TRY(hipMemsetAsync(c->ctrl, 0, sizeof(bq::Ctrl) * MAX_Q, s));
    c->dirty = false;
    return BQ_OK;
}

Queue ctx_queue(const sssp_ctx* c) {
    Queue q;
    q.slots = (decltype(q.slots))c->slots;
    q.ctrl = (decltype(q.ctrl))c->ctrl;
    q.sig = (decltype(q.sig))c->ctrl;
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
// (2 waves) per 8K units of n + m/16, a power of two between 4 and the
// co-resident maximum. More waves than the work can feed only add traffic on
// the queue's hot lines and extra relaxations (labels scanned before they
// settle); sssp_autotune measures instead of guessing.
int default_grid(int n, long long m, int max_grid) {
    // one two-wave workgroup per 8K units of n + m/16
    const unsigned long long units = (unsigned long long)n + (unsigned long long)m / 16ull;
    int g = 4;
    while ((unsigned long long)g * 2ull * 8192ull <= units && g * 2 <= max_grid) g *= 2;
    return g < max_grid ? g : max_grid;
}

// Graphs with fewer than SHORT_ROW_DEGREE edges per vertex on average
// (meshes, road networks) are solved by k_solve_short, which scans
// SHORT_ROW_UNROLL edges per lane per step instead of U: their batches hold
// a few hundred edges, one step of either size, and the shorter step issues
// about half the scan instructions, which is what a batch cycle on such
// graphs (a chain of dependent hops) waits for. 64x64 grid 1.12-1.13 ->
// 1.04-1.06 ms, 2048^2 road mesh 39.7 -> 38.8 ms; an RMAT graph of scale 20
// (16 edges per vertex) needs twice the steps and was 12 % slower with it.
constexpr int SHORT_ROW_UNROLL = 4;
constexpr long long SHORT_ROW_DEGREE = 6;
bool short_rows(long long n, long long m) { return m < SHORT_ROW_DEGREE * n; }

// Co-resident workgroups of k_solve<B> and k_solve_short<B> (slot 0, 1, 2
// for B = 64, 128, 256): the smaller of the two, so that either may be
// launched on a grid of this size.
template <int B>
bq_status occupancy_of_solve(int* per_cu) {
    int a = 0, b = 0;
    BQ_HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&a, k_solve<B>, SOLVE_WG_ONE, 0));
    BQ_HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &b, k_solve_short<B, SHORT_ROW_UNROLL>, SOLVE_WG_ONE, 0));
    *per_cu = a < b ? a : b;
    if (*per_cu < 1) *per_cu = 1;
    return BQ_OK;
}

template <int B>
bq_status solve_max_grid(sssp_ctx* c, int slot, int* out) {
    int& per_cu = c->solve_per_cu[slot];
    if (per_cu == 0) {
        bq_status st = occupancy_of_solve<B>(&per_cu);
        if (st != BQ_OK) return st;
    }
    *out = per_cu * bqh::device_cus();
    return BQ_OK;
}

bq_status max_grid_for(sssp_ctx* c, int batch, int* out) {
    switch (batch) {
        case 1: return solve_max_grid<64>(c, 0, out);
        case 2: return solve_max_grid<128>(c, 1, out);
        default: return solve_max_grid<256>(c, 2, out);
    }
}

bq_status launch_solve(const SolveArgs& args, int batch, int grid, hipStream_t s) {
    constexpr int SU = SHORT_ROW_UNROLL;
    const bool sr = short_rows((long long)args.n, (long long)args.m);
    const dim3 g(grid), b(SOLVE_WG_ONE);
    switch (batch) {
        case 1:
            if (sr) hipLaunchKernelGGL((k_solve_short<64, SU>), g, b, 0, s, args);
            else hipLaunchKernelGGL(k_solve<64>, g, b, 0, s, args);
            break;
        case 2:
            if (sr) hipLaunchKernelGGL((k_solve_short<128, SU>), g, b, 0, s, args);
            else hipLaunchKernelGGL(k_solve<128>, g, b, 0, s, args);
            break;
        default:
            if (sr) hipLaunchKernelGGL((k_solve_short<256, SU>), g, b, 0, s, args);
            else hipLaunchKernelGGL(k_solve<256>, g, b, 0, s, args);
            break;
    }
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
    if (hipMalloc(&c->slots, sizeof(unsigned long long) * cap * MAX_Q) != hipSuccess ||
        hipMalloc(&c->trace, sizeof(unsigned long long) * 4 * TRACE_CAP) != hipSuccess ||
        hipHostMalloc(&c->h_trace, sizeof(unsigned long long) * 4 * TRACE_CAP,
                      hipHostMallocDefault) != hipSuccess ||
        hipMalloc(&c->ctrl, sizeof(bq::Ctrl) * MAX_Q) != hipSuccess ||
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
    if (reps < 1) reps = 5;
    bq_launch L = {};
    if (base) L = *base;
    L.flags &= ~(uint32_t)(BQ_F_TRACE | BQ_F_VALIDATE);
    int max_grid = 0;
    {
        bq_status st = max_grid_for(c, 1, &max_grid);
        if (st != BQ_OK) return st;
    }
    double best = 1e300;
    bq_launch bestL = L;
    auto trial = [&](int wgs, int b, double* out_ms, int chunk = -1, int seg = -1) -> bq_status {
        bq_launch t = L;
        t.wg_count = wgs;
        t.ticket_batch = b;
        if (chunk >= 0) t.row_chunk = chunk;
        if (seg >= 0) t.segments = seg;
        // the median of the runs: the work of an asynchronous solve varies
        // from run to run, and a lucky minimum would pick a shape that is
        // slower on average
        std::vector<double> ts;
        for (int r = 0; r < reps; ++r) {
            int32_t neg = 0;
            bq_status st = sssp_bf(c, n, m, d_offsets, d_cols, d_w, src, d_dist, nullptr, &neg,
                                   &t, stream);
            if (st != BQ_OK) return st;
            ts.push_back(c->last.ms);
        }
        std::sort(ts.begin(), ts.end());
        const double med = (ts[(ts.size() - 1) / 2] + ts[ts.size() / 2]) / 2.0;
        *out_ms = med;
        // a new shape must beat the incumbent by 3 % to replace it
        if (med < best * (best < 1e300 ? 0.97 : 1.0)) {
            best = med;
            bestL = t;
        }
        return BQ_OK;
    };
    // Order of work: one FIFO per home (the method as the paper runs it) or
    // near / far buckets. One series of each at the default grid picks the
    // family the rest of the search tunes: on a large-diameter graph the
    // buckets save most relabels, on a power-law graph they only add work.
    // The bucket family is timed at a step of a quarter of max |w|.
    constexpr int BUCKET_FAMILY_WIDTH = 4;
    if (L.bucket_width == 0) {
        const int g0 = default_grid(n, (long long)m, max_grid);
        std::vector<double> med(2);
        for (int fam = 0; fam < 2; ++fam) {
            bq_launch t = L;
            t.wg_count = g0;
            t.bucket_width = fam ? BUCKET_FAMILY_WIDTH : 0;
            std::vector<double> ts;
            for (int r = 0; r < (reps < 3 ? reps : 3); ++r) {
                int32_t neg = 0;
                bq_status st = sssp_bf(c, n, m, d_offsets, d_cols, d_w, src, d_dist, nullptr,
                                       &neg, &t, stream);
                if (st != BQ_OK) return st;
                ts.push_back(c->last.ms);
            }
            std::sort(ts.begin(), ts.end());
            med[fam] = ts[ts.size() / 2];
        }
        if (med[1] < 0.8 * med[0]) {
            L.bucket_width = BUCKET_FAMILY_WIDTH;
            bestL = L;
        }
    }
    // workgroup count: powers of two upwards until clearly past the minimum
    int best_wgs = 4;
    for (int wgs = 4; wgs <= max_grid; wgs *= 2) {
        double ms = 0;
        bq_status st = trial(wgs, 1, &ms);
        if (st != BQ_OK) return st;
        if (bestL.wg_count == wgs) best_wgs = wgs;
        if (ms > 2.0 * best && wgs >= 4 * best_wgs) break;
        if (wgs * 2 > max_grid && wgs != max_grid) {
            st = trial(max_grid, 1, &ms);
            if (st != BQ_OK) return st;
        }
    }
    const bq_launch pow2L = bestL;  // the best power-of-two count, defaults otherwise
    // counts between the powers of two around the best
    for (int wgs : {best_wgs * 3 / 4, best_wgs * 3 / 2}) {
        if (wgs < 1 || wgs > max_grid || wgs == best_wgs) continue;
        double ms = 0;
        bq_status st = trial(wgs, 1, &ms);
        if (st != BQ_OK) return st;
    }
    best_wgs = bestL.wg_count;
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
        for (int chunk : {64, 256}) {
            double ms = 0;
            bq_status st = trial(cur.wg_count, cur.ticket_batch, &ms, chunk);
            if (st != BQ_OK) return st;
        }
    }
    // queue segments at the best shape: one queue, or 2 / 4 instead of the
    // default (one per XCD)
    {
        const bq_launch cur = bestL;
        for (int seg : {1, 2, 4}) {
            if (seg >= cur.wg_count) continue;
            double ms = 0;
            bq_status st = trial(cur.wg_count, cur.ticket_batch, &ms, cur.row_chunk, seg);
            if (st != BQ_OK) return st;
        }
    }
    // other bucket widths at the best shape, for the bucket family:
    // threshold steps of 1/16, 1/8 and 1 max |w|
    if (bestL.bucket_width > 0) {
        const bq_launch cur = bestL;
        for (int bw : {1, 2, 16}) {
            L.bucket_width = bw;
            double ms = 0;
            bq_status st = trial(cur.wg_count, cur.ticket_batch, &ms, cur.row_chunk, cur.segments);
            if (st != BQ_OK) return st;
        }
        L.bucket_width = cur.bucket_width;
    }
    // confirmation: the winner against the best power-of-two count with
    // default settings, alternating runs, so that one lucky series cannot
    // pick a shape that is slower on average
    if (memcmp(&bestL, &pow2L, sizeof bestL) != 0) {
        std::vector<double> ta, tb;
        for (int r = 0; r < 2 * reps; ++r) {
            for (int side = 0; side < 2; ++side) {
                int32_t neg = 0;
                bq_launch t = side ? pow2L : bestL;
                bq_status st = sssp_bf(c, n, m, d_offsets, d_cols, d_w, src, d_dist, nullptr,
                                       &neg, &t, stream);
                if (st != BQ_OK) return st;
                (side ? tb : ta).push_back(c->last.ms);
            }
        }
        std::sort(ta.begin(), ta.end());
        std::sort(tb.begin(), tb.end());
        const double ma = ta[ta.size() / 2], mb = tb[tb.size() / 2];
        if (mb <= ma) {
            bestL = pow2L;
            best = mb;
        } else {
            best = ma;
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
        hipLaunchKernelGGL(k_validate_csr,
                           dim3(grid_for((int)(m > n ? (m > INT_MAX ? INT_MAX : m) : n))),
                           dim3(256), 0, s, (const long long*)d_offsets, (const int*)d_cols, n,
                           (long long)m, &c->ctrl->aux[3].v);
        BQ_HIP_TRY(hipGetLastError());
        unsigned long long bad = 0;
        BQ_HIP_TRY(hipMemcpyAsync(&bad, &c->ctrl->aux[3].v, 8, hipMemcpyDeviceToHost, s));
        BQ_HIP_TRY(hipStreamSynchronize(s));
        if (bad) return BQ_EINVAL;
    }
    int max_grid = 0;
    {
        bq_status st = max_grid_for(c, L.batch, &max_grid);
        if (st != BQ_OK) return st;
    }
    int grid = L.wg_count > 0 ? L.wg_count : default_grid(n, (long long)m, max_grid);
    if (grid > max_grid) grid = max_grid;  // all waves co-resident
    int nseg = L.segments > 0 ? L.segments : (grid < (int)MAX_SEG ? grid : (int)MAX_SEG);
    if (nseg > (int)MAX_SEG) return BQ_EINVAL;
    if (L.flags & BQ_F_TRACE) nseg = 1;  // the timeline follows one queue
    if (L.bucket_width < 0) return BQ_EINVAL;
    const unsigned shift = key_shift(n);
    SolveArgs a;
    a.q = q;
    a.off = (decltype(a.off))d_offsets;
    a.col = (decltype(a.col))d_cols;
    a.w = (decltype(a.w))d_w;
    a.key = (decltype(a.key))d_dist;
    a.chunk_owner = (decltype(a.chunk_owner))c->chunk_owner;
    a.wrange = (decltype(a.wrange))c->wrange;
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
    a.bwd = (L.flags & BQ_F_BWD) ? 1u : 0u;
    a.nseg = (unsigned)nseg;
    a.bucket_width = L.bucket_width;
    a.nq = (L.bucket_width > 0 ? 3u : 2u) * (unsigned)nseg;
    a.neginf = (L.flags & BQ_F_NEGINF) ? 1u : 0u;
    a.fan_bulk = 0u;
    a.tcol = nullptr;
    a.tw = nullptr;
    a.orig = nullptr;
    a.pos = nullptr;
    if (L.flags & BQ_F_TRACE) {
        // about 256 samples per n + m/C items of work
        unsigned long long unit = (unsigned long long)n + ((unsigned long long)m >> clog);
        unsigned sh = 0;
        while ((1ull << (sh + 8)) < unit) ++sh;
        a.trace = (decltype(a.trace))c->trace;
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
    BQ_HIP_TRY(hipEventRecord(c->evs0, s));
    {
        bq_status st = launch_solve(a, L.batch, grid, s);
        if (st != BQ_OK) return st;
    }
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
    c->last.wg_size = SOLVE_WG_ONE;
    const unsigned long long err = h->error.v;
    const bool neg = h->negcycle.v != 0ull;
    if (err != 0ull || h->abort.v != 0ull) c->dirty = true;  // queue not quiescent
    if (err == bq::ERR_RANGE) return BQ_ERANGE;
    if (err == bq::ERR_FULL) return BQ_EOVERFLOW;
    if (err != 0ull) return BQ_ETIMEOUT;
    *h_neg_cycle = neg ? 1 : 0;
    return BQ_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// sssp_bf_noalloc: sssp_bf for callers that cannot allocate device memory
// ---------------------------------------------------------------------------
// The workspace of one call (control blocks, weight-range partials, chunk
// table, queue slots) lives in the file-scope device array `scratch`: the
// code object reserves it on every device the library runs on, for the
// life of the process. Host code must not pass the array's name to a kernel
// (that is a host-side stand-in, not a device address): the device address
// comes from hipGetSymbolAddress, once per device, with that device
// current, and is kept per device in g_scratch.
namespace {

constexpr unsigned long long NOALLOC_SCRATCH_BYTES = 128ull << 20;
__device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
unsigned char* g_scratch[NOALLOC_MAX_DEVICES];      // device address per device
int g_scratch_per_cu[NOALLOC_MAX_DEVICES][3];        // occupancy of k_solve<64/128/256>

inline unsigned long long round256(unsigned long long x) { return (x + 255ull) & ~255ull; }

// Device address of `scratch` on the current device (looked up on the first
// call there).
bq_status scratch_of_current_device(int* dev_out, unsigned char** out) {
    int dev = 0;
    BQ_HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return BQ_EINVAL;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        BQ_HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return BQ_EHIP;
        g_scratch[dev] = (unsigned char*)p;
    }
    *dev_out = dev;
    *out = g_scratch[dev];
    return BQ_OK;
}

bq_status noalloc_max_grid(int dev, int batch, int* out) {
    const int slot = batch == 1 ? 0 : (batch == 2 ? 1 : 2);
    int per_cu = 0;
    {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        per_cu = g_scratch_per_cu[dev][slot];
    }
    if (per_cu == 0) {
        bq_status st = batch == 1 ? occupancy_of_solve<64>(&per_cu)
                                  : (batch == 2 ? occupancy_of_solve<128>(&per_cu)
                                                : occupancy_of_solve<256>(&per_cu));
        if (st != BQ_OK) return st;
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        g_scratch_per_cu[dev][slot] = per_cu;
    }
    *out = per_cu * bqh::device_cus();
    return BQ_OK;
}

// zero `words` 64-bit words (a kernel rather than a memset, so that the
// sequence stays a plain chain of kernels)
__global__ void k_zero_words(unsigned long long* p, unsigned long long words) {
    const unsigned long long stride = (unsigned long long)gridDim.x * blockDim.x;
    for (unsigned long long i = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x;
         i < words; i += stride)
        p[i] = 0ull;
}

}  // namespace

extern "C" bq_status sssp_bf_noalloc(int32_t n, int64_t m, const int64_t* d_offsets,
                                     const int32_t* d_cols, const int32_t* d_w, int32_t src,
                                     int64_t* d_dist, int32_t* d_pred, int32_t* h_neg_cycle,
                                     const bq_launch* launch, void* stream) {
    if (!d_offsets || !d_dist || !h_neg_cycle) return BQ_EINVAL;
    if (n < 1 || m < 0 || src < 0 || src >= n) return BQ_EINVAL;
    if (m > 0 && (!d_cols || !d_w)) return BQ_EINVAL;
    unsigned clog = DEFAULT_CHUNK_LOG;
    if (launch && launch->row_chunk > 0) {
        const int rc = launch->row_chunk;
        if (rc & (rc - 1)) return BQ_EINVAL;
        clog = bqh::log2_exact((unsigned long long)rc);
        if (clog < MIN_CHUNK_LOG || clog > MAX_CHUNK_LOG) return BQ_EINVAL;
    }
    if ((unsigned long long)n + ((unsigned long long)m >> clog) + 1ull >= 0xFFFFFFFFull)
        return BQ_EINVAL;
    bqh::Launch L = bqh::resolve(launch, 0);
    if (L.batch != 1 && L.batch != 2 && L.batch != 4) return BQ_EINVAL;
    if (L.flags & BQ_F_TRACE) return BQ_EINVAL;  // the timeline needs a context
    hipStream_t s = bqh::as_stream(stream);
    int dev = 0;
    unsigned char* base = nullptr;
    {
        bq_status st = scratch_of_current_device(&dev, &base);
        if (st != BQ_OK) return st;
    }
    int max_grid = 0;
    {
        bq_status st = noalloc_max_grid(dev, L.batch, &max_grid);
        if (st != BQ_OK) return st;
    }
    int grid = L.wg_count > 0 ? L.wg_count : default_grid(n, (long long)m, max_grid);
    if (grid > max_grid) grid = max_grid;
    int nseg = L.segments > 0 ? L.segments : (grid < (int)MAX_SEG ? grid : (int)MAX_SEG);
    if (nseg > (int)MAX_SEG) return BQ_EINVAL;
    if (L.bucket_width < 0) return BQ_EINVAL;
    const unsigned nq = (L.bucket_width > 0 ? 3u : 2u) * (unsigned)nseg;

    // layout of this call in the scratch array: control blocks of all MAX_Q
    // queues (k_init reads every block), weight-range partials, chunk
    // table, then the slots of the nq queues it uses (each sized as in
    // sssp_ctx_create: 2 * pow2(n + m / 64 + 1), at least 4096)
    const unsigned long long need =
        (unsigned long long)n + ((unsigned long long)m >> MIN_CHUNK_LOG) + 1ull;
    unsigned long long cap = 4096ull;
    while (cap < 2ull * need) cap <<= 1;
    const unsigned long long ctrl_bytes = round256(sizeof(bq::Ctrl) * MAX_Q);
    const unsigned long long wr_bytes = round256(sizeof(int) * 2 * INIT_MAX_BLOCKS);
    const unsigned long long ch_bytes =
        round256(sizeof(unsigned) * (((unsigned long long)m >> clog) + 1ull));
    const unsigned long long slot_words = (unsigned long long)nq * cap;
    const unsigned long long total = ctrl_bytes + wr_bytes + ch_bytes + 8ull * slot_words;
    if (cap > (1ull << 31) || total > NOALLOC_SCRATCH_BYTES) return BQ_EBUSY;
    bq::Ctrl* ctrl = (bq::Ctrl*)base;
    int* wrange = (int*)(base + ctrl_bytes);
    unsigned* chunk_owner = (unsigned*)(base + ctrl_bytes + wr_bytes);
    unsigned long long* slots = (unsigned long long*)(base + ctrl_bytes + wr_bytes + ch_bytes);

    // the array keeps the previous call's contents: clear the control
    // blocks and the slots this call uses
    hipLaunchKernelGGL(k_zero_words, dim3(64), dim3(256), 0, s, (unsigned long long*)ctrl,
                       (unsigned long long)(ctrl_bytes / 8));
    BQ_HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_zero_words, dim3(grid_for((int)std::min<unsigned long long>(
                                          slot_words / 8, (unsigned long long)INT_MAX))),
                       dim3(256), 0, s, slots, slot_words);
    BQ_HIP_TRY(hipGetLastError());

    Queue q;
    q.slots = (decltype(q.slots))slots;
    q.ctrl = (decltype(q.ctrl))ctrl;
    q.sig = (decltype(q.sig))ctrl;
    q.logN = bqh::log2_exact(cap);
    q.pad = 0;
    q.N = cap;
    if (L.flags & BQ_F_VALIDATE) {
        hipLaunchKernelGGL(k_validate_csr,
                           dim3(grid_for((int)(m > n ? (m > INT_MAX ? INT_MAX : m) : n))),
                           dim3(256), 0, s, (const long long*)d_offsets, (const int*)d_cols, n,
                           (long long)m, &ctrl->aux[3].v);
        BQ_HIP_TRY(hipGetLastError());
        unsigned long long bad = 0;
        BQ_HIP_TRY(hipMemcpyAsync(&bad, &ctrl->aux[3].v, 8, hipMemcpyDeviceToHost, s));
        BQ_HIP_TRY(hipStreamSynchronize(s));
        if (bad) return BQ_EINVAL;
    }
    const unsigned shift = key_shift(n);
    SolveArgs a;
    a.q = q;
    a.off = (decltype(a.off))d_offsets;
    a.col = (decltype(a.col))d_cols;
    a.w = (decltype(a.w))d_w;
    a.key = (decltype(a.key))d_dist;
    a.chunk_owner = (decltype(a.chunk_owner))chunk_owner;
    a.wrange = (decltype(a.wrange))wrange;
    a.n = n;
    a.src = src;
    a.m = (long long)m;
    a.shift = shift;
    a.chunk_log = clog;
    a.limit = L.limit;
    a.deadline = 10ull * L.limit;
    a.trace = nullptr;
    a.trace_shift = 0;
    a.trace_cap = 0;
    a.bwd = (L.flags & BQ_F_BWD) ? 1u : 0u;
    a.nseg = (unsigned)nseg;
    a.bucket_width = L.bucket_width;
    a.nq = (L.bucket_width > 0 ? 3u : 2u) * (unsigned)nseg;
    a.neginf = (L.flags & BQ_F_NEGINF) ? 1u : 0u;
    a.fan_bulk = 0u;
    a.tcol = nullptr;
    a.tw = nullptr;
    a.orig = nullptr;
    a.pos = nullptr;
    {
        const long long big = m > n ? m : n;
        long long blocks = (big + (long long)INIT_WG * 8 - 1) / ((long long)INIT_WG * 8);
        if (blocks < 1) blocks = 1;
        if (blocks > INIT_MAX_BLOCKS) blocks = INIT_MAX_BLOCKS;
        hipLaunchKernelGGL(k_init, dim3((unsigned)blocks), dim3(INIT_WG), 0, s, q,
                           (long long*)d_dist, n, src, shift, (const int*)d_w, (long long)m,
                           wrange);
        BQ_HIP_TRY(hipGetLastError());
    }
    {
        bq_status st = launch_solve(a, L.batch, grid, s);
        if (st != BQ_OK) return st;
    }
    hipLaunchKernelGGL(k_unpack, dim3(grid_for(n)), dim3(256), 0, s, (long long*)d_dist,
                       (int*)d_pred, n, src, shift);
    BQ_HIP_TRY(hipGetLastError());
    unsigned long long words[3] = {0, 0, 0};
    BQ_HIP_TRY(hipMemcpyAsync(&words[0], &ctrl->error.v, 8, hipMemcpyDeviceToHost, s));
    BQ_HIP_TRY(hipMemcpyAsync(&words[1], &ctrl->negcycle.v, 8, hipMemcpyDeviceToHost, s));
    BQ_HIP_TRY(hipMemcpyAsync(&words[2], &ctrl->abort.v, 8, hipMemcpyDeviceToHost, s));
    BQ_HIP_TRY(hipStreamSynchronize(s));
    if (words[0] == bq::ERR_RANGE) return BQ_ERANGE;
    if (words[0] == bq::ERR_FULL) return BQ_EOVERFLOW;
    if (words[0] != 0ull) return BQ_ETIMEOUT;
    *h_neg_cycle = words[1] != 0ull ? 1 : 0;
    return BQ_OK;
}
