// The Broker Queue as a stand-alone concurrent FIFO (Section III.A, Alg. 1)
// and the "Global Mixed" benchmark of Section IV, for gfx950.
//
// Kernels:
//  k_bulk_enqueue  - ENQUEUE of an array of values, wave-aggregated
//  k_bulk_dequeue  - DEQUEUE of up to n values into a compacted array
//  k_bench_mixed   - even workgroups enqueue, odd workgroups dequeue,
//                    concurrently, each lane retrying Full/Empty attempts
#include <hip/hip_runtime.h>
#include <stdio.h>
#include <stdlib.h>

#include "host_common.hpp"

using bq::Queue;

// Partitioned form (the paper's multi-GPU queue of Section III.B and Alg. 2
// on the chip's XCDs): the benchmarks can split the queue into S = 2, 4 or 8
// segments, each a complete Broker Queue over capacity / S slots with its own
// control block. Workgroup i works on segment i mod S (workgroups are
// dispatched to the XCDs in turn), and each segment carries 1/S of the
// operations, as each GPU does in Alg. 2.
constexpr unsigned MAX_QSEG = 8;

struct bq_queue {
    int device;
    uint32_t capacity;
    uint32_t logN;
    unsigned long long* slots;   // [capacity] (ticket << 32 | payload)
    bq::Ctrl* ctrl;              // [MAX_QSEG]; block 0 serves the unsegmented queue
    unsigned long long* scratch;  // device counters for the bench
    hipEvent_t ev0, ev1;
};

namespace {

// `sig`: the control block whose abort / error words stop every segment
__device__ __forceinline__ Queue view(unsigned long long* sl, bq::Ctrl* c, uint32_t logN,
                                      bq::Ctrl* sig) {
    Queue q;
    q.slots = (decltype(q.slots))sl;
    q.ctrl = (decltype(q.ctrl))c;
    q.sig = (decltype(q.sig))sig;
    q.logN = logN;
    q.pad = 0;
    q.N = 1ull << logN;
    return q;
}

// One wave moves one chunk of `cnt` operations (cnt <= 64*b). ENQ: item j
// enqueues vals[first + j] (or first + j when vals is NULL); !ENQ: item j
// dequeues into out[] at an index taken from *n_out (compacted, position
// order within a reservation). Successful items are always a prefix of the
// chunk, so one wave keeps array order.
//
// After a reservation that did not cover the rest of the chunk:
//  - Broker Queue (Alg. 1 ENQUEUE / DEQUEUE): look at head and tail; if the
//    queue is not Full (Empty) the shortfall was transient and the wave tries
//    again at once; if it is, the operations return Full (Empty);
//  - BWD (bwd = true): the single-shot broker check of the Broker Work
//    Distributor returns Full (Empty) at once.
// Operations that returned Full / Empty are retried after a backoff when
// `retry` is set (the benchmark's policy) and given up otherwise.
// Returns the number done; *fails counts Full / Empty returns.
template <bool ENQ>
__device__ unsigned long long chunk_op(const Queue& q, unsigned long long first,
                                       unsigned long long cnt, const int32_t* vals, int32_t* out,
                                       unsigned long long* n_out, int32_t* log,
                                       bool bwd, bool retry, unsigned long long limit,
                                       unsigned long long& spins, unsigned long long& fails,
                                       bool& bad) {
    const int lane = bq::lane_id();
    unsigned long long done = 0;
    int level = 0;
    bq::Watch wd;
    wd.arm(limit);
    while (done < cnt) {
        uint32_t e = 0;
        unsigned long long base = 0, obase = 0;
        if (lane == 0) {
            const uint32_t want = (uint32_t)(cnt - done);
            e = ENQ ? bq::reserve_enqueue(q, want) : bq::reserve_dequeue(q, want);
            if (e) {
                base = bq::add_rlx(ENQ ? &q.ctrl->tail.v : &q.ctrl->head.v, (unsigned long long)e);
                if (!ENQ && n_out) obase = bq::add_rlx(n_out, (unsigned long long)e);
            }
        }
        e = bq::bcast32(e);
        base = bq::bcast64(base);
        obase = bq::bcast64(obase);
        for (uint32_t j0 = 0; j0 < e; j0 += 64) {
            const uint32_t j = j0 + (uint32_t)lane;
            const bool act = j < e;
            const unsigned long long pos = base + j;
            const unsigned long long item = first + done + j;
            if (ENQ) {
                const uint32_t val = act ? (vals ? (uint32_t)vals[item] : (uint32_t)item) : 0u;
                if (!bq::put_slots(q, act, pos, val, limit, spins)) {
                    bad = true;
                    return done;
                }
                if (act && log) log[pos] = (int32_t)val;
            } else {
                uint32_t val = 0;
                if (!bq::read_slots(q, act, pos, val, limit, spins)) {
                    bad = true;
                    return done;
                }
                if (act && out) out[obase + j] = (int32_t)val;
                if (act && log) log[pos] = (int32_t)val;
            }
        }
        done += e;
        if (done == cnt) break;
        bool refused = true;  // BWD: the single-shot check already said Full/Empty
        if (!bwd) {
            bool st = false;
            if (lane == 0) st = ENQ ? bq::looks_full(q) : bq::looks_empty(q);
            refused = bq::bcast32(st) != 0;
        }
        if (refused) {
            ++fails;
            if (!retry) break;
        }
        if (bq::aborted(q)) {
            bad = true;
            break;
        }
        if (wd.expired()) {
            if (lane == 0) bq::raise_error(q, bq::ERR_TIMEOUT);
            bad = true;
            break;
        }
        if (refused) {
            bq::backoff(level);
            if (level < 3) ++level;
        }
    }
    return done;
}

// ENQUEUE (ENQ) or DEQUEUE of n operations, grid-stride over chunks of
// 64*b; every operation makes one attempt (Successful / Full, data / Empty).
// With lseg > 0 the queue is split into 2^lseg segments (see bq_queue):
// workgroup i works on segment i mod 2^lseg, and segment s owns operations
// [s n / 2^lseg, (s+1) n / 2^lseg).
template <bool ENQ>
__global__ void k_bulk(unsigned long long* slots, bq::Ctrl* ctrl, uint32_t logN,
                       const int32_t* vals, int32_t* out, unsigned long long n,
                       unsigned long long* n_ok, unsigned long long* stats,
                       unsigned long long limit, unsigned b, int bwd, unsigned lseg) {
    const unsigned S = 1u << lseg;
    const unsigned seg = blockIdx.x & (S - 1u);
    const Queue q = view(slots + ((unsigned long long)seg << (logN - lseg)), ctrl + seg,
                         logN - lseg, ctrl);
    const unsigned long long wpb = blockDim.x >> 6;
    const unsigned long long waves = (unsigned long long)(gridDim.x >> lseg) * wpb;
    const unsigned long long wave = (unsigned long long)(blockIdx.x >> lseg) * wpb + (threadIdx.x >> 6);
    const unsigned long long per = n >> lseg;  // the host checks n % S == 0
    const unsigned long long lo = per * seg;
    const unsigned long long K = 64ull * b;
    unsigned long long ok = 0, spins = 0, fails = 0;
    bool bad = false;
    for (unsigned long long c = wave; c * K < per && !bad; c += waves) {
        const unsigned long long first = lo + c * K;
        const unsigned long long cnt = (per - c * K) < K ? (per - c * K) : K;
        ok += chunk_op<ENQ>(q, first, cnt, vals, out, n_ok, nullptr, bwd != 0, false, limit, spins,
                            fails, bad);
    }
    if (bq::lane_id() == 0) {
        if (ENQ && ok) bq::add_rlx(n_ok, ok);
        if (stats && fails) bq::add_rlx(&stats[ENQ ? 2 : 3], fails);
        if (stats && ok) bq::add_rlx(&stats[ENQ ? 0 : 1], ok);
    }
}

// Section IV "Global Mixed": even workgroups enqueue, odd dequeue. A wave
// takes chunks of K = 64*b operations (grid-stride over chunks) and moves
// each with as few broker reservations and head/tail tickets as the queue
// state allows; operations that return Full / Empty are retried after a
// backoff until the chunk is done. Enqueue operation i writes value i.
// stats[0..3] = enq_ok, deq_ok, enq_full, deq_empty.
// Partitioned (lseg > 0): workgroup i works on segment s = i mod S and is
// an enqueuer when (i / S) is even; segment s carries operations
// [s n_half / S, (s+1) n_half / S) of each kind, and its logs are the same
// slices of enq_log / deq_log (position P of segment s at index
// s n_half / S + P).
__global__ void k_bench_mixed(unsigned long long* slots, bq::Ctrl* ctrl, uint32_t logN,
                              unsigned long long n_half, int32_t* enq_log, int32_t* deq_log,
                              unsigned long long* stats, unsigned long long limit, unsigned b,
                              int bwd, unsigned lseg) {
    const unsigned S = 1u << lseg;
    const unsigned seg = blockIdx.x & (S - 1u);
    const unsigned rank = blockIdx.x >> lseg;  // workgroup's rank in its segment
    const Queue q = view(slots + ((unsigned long long)seg << (logN - lseg)), ctrl + seg,
                         logN - lseg, ctrl);
    const int wpb = blockDim.x >> 6;
    const unsigned gps = gridDim.x >> lseg;    // the host makes grid a multiple of 2S
    const bool enq = (rank & 1u) == 0u;
    const unsigned long long role_blocks = enq ? (gps + 1u) / 2u : gps / 2u;
    const unsigned long long waves = role_blocks * (unsigned long long)wpb;
    const unsigned long long wave = (unsigned long long)(rank >> 1) * wpb + (threadIdx.x >> 6);
    const unsigned long long per = n_half >> lseg;  // the host checks n_half % S == 0
    const unsigned long long lo = per * seg;
    int32_t* elog = enq_log ? enq_log + lo : nullptr;
    int32_t* dlog = deq_log ? deq_log + lo : nullptr;
    const unsigned long long K = 64ull * b;
    unsigned long long ok = 0, spins = 0, fails = 0;
    bool bad = false;
    for (unsigned long long c = wave; c * K < per && !bad; c += waves) {
        const unsigned long long first = lo + c * K;
        const unsigned long long cnt = (per - c * K) < K ? (per - c * K) : K;
        ok += enq ? chunk_op<true>(q, first, cnt, nullptr, nullptr, nullptr, elog, bwd != 0,
                                   true, limit, spins, fails, bad)
                  : chunk_op<false>(q, first, cnt, nullptr, nullptr, nullptr, dlog, bwd != 0,
                                    true, limit, spins, fails, bad);
    }
    if (bq::lane_id() == 0) {
        if (ok) bq::add_rlx(&stats[enq ? 0 : 1], ok);
        if (fails) bq::add_rlx(&stats[enq ? 2 : 3], fails);
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// host API
// ---------------------------------------------------------------------------
namespace bqh {

static thread_local char g_last_err[256];

void note_hip_error(hipError_t e, const char* what, int line) {
    snprintf(g_last_err, sizeof g_last_err, "%s (line %d): %s", what, line, hipGetErrorString(e));
    if (getenv("BQ_DEBUG")) fprintf(stderr, "bqsssp: %s\n", g_last_err);
}

int device_cus() {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    return cus;
}

Launch resolve(const bq_launch* l, int default_wgs) {
    Launch r;
    r.wg_size = (l && l->wg_size > 0) ? l->wg_size : 256;
    r.wg_count = (l && l->wg_count > 0) ? l->wg_count : default_wgs;
    r.batch = (l && l->ticket_batch > 0) ? l->ticket_batch : 1;
    r.row_chunk = (l && l->row_chunk > 0) ? l->row_chunk : 0;
    r.segments = (l && l->segments > 0) ? l->segments : 0;
    r.bucket_width = l ? l->bucket_width : 0;
    r.flags = l ? l->flags : 0u;
    const unsigned long long us = (l && l->timeout_us) ? l->timeout_us : 2000000ull;
    r.limit = us * 100ull;  // 100 MHz
    return r;
}

}  // namespace bqh

extern "C" {

const char* bq_strerror(bq_status s) {
    switch (s) {
        case BQ_OK: return "ok";
        case BQ_EINVAL: return "invalid argument";
        case BQ_ENOMEM: return "out of device memory";
        case BQ_EHIP: return "HIP runtime error";
        case BQ_ERANGE: return "distances do not fit the packed key (n * max|w| too large)";
        case BQ_ETIMEOUT: return "device watchdog fired";
        case BQ_EOVERFLOW: return "solver queue over capacity (library fault)";
        case BQ_EBUSY: return "object too small for this input";
    }
    return "unknown status";
}

int32_t bq_device_cus(void) { return bqh::device_cus(); }

static bq_status queue_zero(bq_queue* q, hipStream_t s) {
    BQ_HIP_TRY(hipMemsetAsync(q->slots, 0, sizeof(unsigned long long) * q->capacity, s));
    BQ_HIP_TRY(hipMemsetAsync(q->ctrl, 0, sizeof(bq::Ctrl) * MAX_QSEG, s));
    return BQ_OK;
}

// log2 of the benchmark's segment count (launch field `segments`, 0 = 1):
// 1, 2, 4 or 8, each segment at least 64*b slots; -1 if invalid
static int seg_log(const bq_queue* q, const bqh::Launch& L) {
    const int S = L.segments > 0 ? L.segments : 1;
    if (S > (int)MAX_QSEG || (S & (S - 1))) return -1;
    const int lseg = (int)bqh::log2_exact((unsigned long long)S);
    if ((unsigned long long)(q->capacity >> lseg) < 64ull * (unsigned long long)L.batch) return -1;
    return lseg;
}

bq_status bq_create(uint32_t capacity, uint32_t flags, void* stream, bq_queue** out) {
    (void)flags;
    if (!out || capacity < 64u || (capacity & (capacity - 1u)) != 0u) return BQ_EINVAL;
    *out = nullptr;
    bq_queue* q = (bq_queue*)calloc(1, sizeof(bq_queue));
    if (!q) return BQ_ENOMEM;
    BQ_HIP_TRY(hipGetDevice(&q->device));
    q->capacity = capacity;
    q->logN = bqh::log2_exact(capacity);
    if (hipMalloc(&q->slots, sizeof(unsigned long long) * capacity) != hipSuccess ||
        hipMalloc(&q->ctrl, sizeof(bq::Ctrl) * MAX_QSEG) != hipSuccess ||
        hipMalloc(&q->scratch, 4096) != hipSuccess) {
        bq_destroy(q);
        return BQ_ENOMEM;
    }
    BQ_HIP_TRY(hipEventCreate(&q->ev0));
    BQ_HIP_TRY(hipEventCreate(&q->ev1));
    bq_status st = queue_zero(q, bqh::as_stream(stream));
    if (st != BQ_OK) {
        bq_destroy(q);
        return st;
    }
    BQ_HIP_TRY(hipStreamSynchronize(bqh::as_stream(stream)));
    *out = q;
    return BQ_OK;
}

bq_status bq_destroy(bq_queue* q) {
    if (!q) return BQ_OK;
    (void)hipDeviceSynchronize();
    if (q->slots) (void)hipFree(q->slots);
    if (q->ctrl) (void)hipFree(q->ctrl);
    if (q->scratch) (void)hipFree(q->scratch);
    if (q->ev0) (void)hipEventDestroy(q->ev0);
    if (q->ev1) (void)hipEventDestroy(q->ev1);
    free(q);
    return BQ_OK;
}

bq_status bq_reset(bq_queue* q, void* stream) {
    if (!q) return BQ_EINVAL;
    bq_status st = queue_zero(q, bqh::as_stream(stream));
    if (st != BQ_OK) return st;
    BQ_HIP_TRY(hipStreamSynchronize(bqh::as_stream(stream)));
    return BQ_OK;
}

bq_status bq_counters(bq_queue* q, void* stream, uint64_t* h_head, uint64_t* h_tail,
                      int64_t* h_count) {
    if (!q) return BQ_EINVAL;
    hipStream_t s = bqh::as_stream(stream);
    unsigned long long v[3];
    BQ_HIP_TRY(hipMemcpyAsync(&v[0], &q->ctrl->head.v, 8, hipMemcpyDeviceToHost, s));
    BQ_HIP_TRY(hipMemcpyAsync(&v[1], &q->ctrl->tail.v, 8, hipMemcpyDeviceToHost, s));
    BQ_HIP_TRY(hipMemcpyAsync(&v[2], &q->ctrl->count.v, 8, hipMemcpyDeviceToHost, s));
    BQ_HIP_TRY(hipStreamSynchronize(s));
    if (h_head) *h_head = v[0];
    if (h_tail) *h_tail = v[1];
    if (h_count) *h_count = (int64_t)v[2];
    return BQ_OK;
}

// error words of every segment (the unsegmented queue uses block 0)
static bq_status check_error_and_reset(bq_queue* q, hipStream_t s) {
    unsigned long long errs[MAX_QSEG];
    for (unsigned i = 0; i < MAX_QSEG; ++i)
        BQ_HIP_TRY(hipMemcpyAsync(&errs[i], &q->ctrl[i].error.v, 8, hipMemcpyDeviceToHost, s));
    BQ_HIP_TRY(hipStreamSynchronize(s));
    unsigned long long err = 0;
    for (unsigned i = 0; i < MAX_QSEG; ++i) err |= errs[i];
    if (err != 0ull) {
        queue_zero(q, s);
        BQ_HIP_TRY(hipStreamSynchronize(s));
        return BQ_ETIMEOUT;
    }
    return BQ_OK;
}

static bq_status bulk(bq_queue* q, bool enq, const int32_t* vals, int32_t* out, uint64_t n,
                      uint64_t* d_n_ok, unsigned long long* d_stats, const bq_launch* launch,
                      hipStream_t s, bool reset_count, unsigned lseg) {
    bqh::Launch L = bqh::resolve(launch, 4 * bqh::device_cus());
    if (L.wg_size % 64 || L.wg_size > 1024 || L.batch < 1 ||
        64ull * (unsigned long long)L.batch > (unsigned long long)(q->capacity >> lseg))
        return BQ_EINVAL;
    if (reset_count) BQ_HIP_TRY(hipMemsetAsync(d_n_ok, 0, 8, s));
    if (n) {
        const unsigned long long S = 1ull << lseg;
        const unsigned long long K = 64ull * (unsigned long long)L.batch;
        const unsigned long long chunks = S * (((n >> lseg) + K - 1) / K);
        const unsigned long long wpb = (unsigned long long)(L.wg_size / 64);
        unsigned long long g = (chunks + wpb - 1) / wpb;
        if (g > (unsigned long long)L.wg_count) g = (unsigned long long)L.wg_count;
        g -= g % S;  // every segment gets the same number of workgroups
        if (g < S) g = S;
        const int bwd = (L.flags & BQ_F_BWD) ? 1 : 0;
        if (enq)
            hipLaunchKernelGGL(k_bulk<true>, dim3((unsigned)g), dim3(L.wg_size), 0, s, q->slots,
                               q->ctrl, q->logN, vals, (int32_t*)nullptr, (unsigned long long)n,
                               (unsigned long long*)d_n_ok, d_stats, L.limit,
                               (unsigned)L.batch, bwd, lseg);
        else
            hipLaunchKernelGGL(k_bulk<false>, dim3((unsigned)g), dim3(L.wg_size), 0, s, q->slots,
                               q->ctrl, q->logN, (const int32_t*)nullptr, out,
                               (unsigned long long)n, (unsigned long long*)d_n_ok, d_stats,
                               L.limit, (unsigned)L.batch, bwd, lseg);
        BQ_HIP_TRY(hipGetLastError());
    }
    return BQ_OK;
}

bq_status bq_enqueue(bq_queue* q, const int32_t* d_vals, uint64_t n, uint64_t* d_n_ok,
                     const bq_launch* launch, void* stream) {
    if (!q || !d_n_ok || (n && !d_vals)) return BQ_EINVAL;
    hipStream_t s = bqh::as_stream(stream);
    bq_status st = bulk(q, true, d_vals, nullptr, n, d_n_ok, nullptr, launch, s, true, 0);
    if (st != BQ_OK) return st;
    return check_error_and_reset(q, s);
}

bq_status bq_dequeue(bq_queue* q, int32_t* d_out, uint64_t n, uint64_t* d_n_ok,
                     const bq_launch* launch, void* stream) {
    if (!q || !d_n_ok || (n && !d_out)) return BQ_EINVAL;
    hipStream_t s = bqh::as_stream(stream);
    bq_status st = bulk(q, false, nullptr, d_out, n, d_n_ok, nullptr, launch, s, true, 0);
    if (st != BQ_OK) return st;
    return check_error_and_reset(q, s);
}

bq_status bq_bench_enqdeq(bq_queue* q, uint64_t n_ops, const bq_launch* launch,
                          bq_bench_stats* h_enq, bq_bench_stats* h_deq, void* stream) {
    if (!q || n_ops < 2 || (n_ops & 1ull) || n_ops / 2 > 0x7fffffffull || !h_enq || !h_deq)
        return BQ_EINVAL;
    hipStream_t s = bqh::as_stream(stream);
    const int lseg = seg_log(q, bqh::resolve(launch, 0));
    if (lseg < 0 || (n_ops / 2) % (1ull << lseg)) return BQ_EINVAL;
    bq_status st = queue_zero(q, s);
    if (st != BQ_OK) return st;
    BQ_HIP_TRY(hipMemsetAsync(q->scratch, 0, 128, s));
    unsigned long long* stats = q->scratch;
    unsigned long long* cursor = q->scratch + 8;
    const unsigned long long half = n_ops / 2;
    hipEvent_t e0 = q->ev0, e1 = q->ev1;
    hipEvent_t e2;
    BQ_HIP_TRY(hipEventCreate(&e2));
    BQ_HIP_TRY(hipEventRecord(e0, s));
    st = bulk(q, true, nullptr, nullptr, half, (uint64_t*)cursor, stats, launch, s, false,
              (unsigned)lseg);
    if (st != BQ_OK) return st;
    BQ_HIP_TRY(hipEventRecord(e1, s));
    st = bulk(q, false, nullptr, nullptr, half, (uint64_t*)(cursor + 1), stats, launch, s,
              false, (unsigned)lseg);
    if (st != BQ_OK) return st;
    BQ_HIP_TRY(hipEventRecord(e2, s));
    unsigned long long h[4];
    BQ_HIP_TRY(hipMemcpyAsync(h, stats, sizeof h, hipMemcpyDeviceToHost, s));
    st = check_error_and_reset(q, s);
    float ms1 = 0.f, ms2 = 0.f;
    BQ_HIP_TRY(hipEventElapsedTime(&ms1, e0, e1));
    BQ_HIP_TRY(hipEventElapsedTime(&ms2, e1, e2));
    (void)hipEventDestroy(e2);
    *h_enq = bq_bench_stats{h[0], 0, h[2], 0, ms1};
    *h_deq = bq_bench_stats{0, h[1], 0, h[3], ms2};
    return st;
}

bq_status bq_bench_mixed(bq_queue* q, uint64_t n_ops, const bq_launch* launch,
                         int32_t* d_enq_log, int32_t* d_deq_log, bq_bench_stats* h_out,
                         int32_t* h_enq_waves, void* stream) {
    if (!q || n_ops < 2 || (n_ops & 1ull) || n_ops / 2 > 0x7fffffffull) return BQ_EINVAL;
    hipStream_t s = bqh::as_stream(stream);
    bqh::Launch L = bqh::resolve(launch, 0);
    if (L.wg_size % 64 || L.wg_size > 1024) return BQ_EINVAL;
    if (L.batch < 1 || 64ull * (unsigned long long)L.batch > q->capacity) return BQ_EINVAL;
    const int lseg = seg_log(q, L);
    if (lseg < 0 || (n_ops / 2) % (1ull << lseg)) return BQ_EINVAL;
    const int S2 = 2 << lseg;  // each segment needs an enqueuer and a dequeuer workgroup
    // co-resident grid: enqueuers spin on Full until dequeuers run, so all
    // workgroups must be resident together. The grid is clamped to what the
    // occupancy calculator says fits, as for the persistent solver, and a
    // wait that never ended would still stop at the watchdog (BQ_ETIMEOUT).
    int per_cu = 0;
    BQ_HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_bench_mixed, L.wg_size, 0));
    const int max_grid = per_cu * bqh::device_cus();
    int grid = L.wg_count > 0 ? L.wg_count : max_grid;
    if (grid > max_grid) grid = max_grid;
    grid -= grid % S2;
    if (grid < S2) return BQ_EINVAL;
    // start from an empty, zeroed queue (outside the timed region)
    bq_status st = queue_zero(q, s);
    if (st != BQ_OK) return st;
    BQ_HIP_TRY(hipMemsetAsync(q->scratch, 0, 64, s));
    unsigned long long n_half = n_ops / 2ull;
    int32_t* el = d_enq_log;
    int32_t* dl = d_deq_log;
    unsigned long long* stats = q->scratch;
    unsigned long long* sl = q->slots;
    bq::Ctrl* ct = q->ctrl;
    uint32_t lg = q->logN;
    unsigned long long lim = L.limit;
    unsigned bb = (unsigned)L.batch;
    int bwd = (L.flags & BQ_F_BWD) ? 1 : 0;
    unsigned ls = (unsigned)lseg;
    void* args[] = {&sl, &ct, &lg, &n_half, &el, &dl, &stats, &lim, &bb, &bwd, &ls};
    BQ_HIP_TRY(hipEventRecord(q->ev0, s));
    BQ_HIP_TRY(hipLaunchKernel((const void*)k_bench_mixed, dim3(grid), dim3(L.wg_size), args, 0,
                               s));
    BQ_HIP_TRY(hipEventRecord(q->ev1, s));
    unsigned long long h[4];
    BQ_HIP_TRY(hipMemcpyAsync(h, q->scratch, sizeof h, hipMemcpyDeviceToHost, s));
    st = check_error_and_reset(q, s);
    float ms = 0.f;
    BQ_HIP_TRY(hipEventElapsedTime(&ms, q->ev0, q->ev1));
    if (h_out) {
        h_out->enq_ok = h[0];
        h_out->deq_ok = h[1];
        h_out->enq_full = h[2];
        h_out->deq_empty = h[3];
        h_out->ms = ms;
    }
    if (h_enq_waves) *h_enq_waves = (grid / 2) * (L.wg_size / 64);
    return st;
}

}  // extern "C"
