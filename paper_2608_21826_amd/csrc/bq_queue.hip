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

struct bq_queue {
    int device;
    uint32_t capacity;
    uint32_t logN;
    unsigned long long* slots;   // [capacity] (ticket << 32 | payload)
    bq::Ctrl* ctrl;
    unsigned long long* scratch;  // device counters for the bench
    hipEvent_t ev0, ev1;
};

namespace {

__device__ __forceinline__ Queue view(unsigned long long* sl, bq::Ctrl* c, uint32_t logN) {
    Queue q;
    q.slots = sl;
    q.ctrl = c;
    q.logN = logN;
    q.pad = 0;
    q.N = 1ull << logN;
    return q;
}

// One wave enqueues the values of its active lanes (Alg. 1 ENQUEUE, all
// lanes at once). Lanes whose reservation fails retry while the queue is not
// Full; with `give_up_on_full` they stop (result Full), otherwise they retry
// after a backoff until they succeed (the benchmark's retry policy).
// Returns per-lane: 1 success, 0 Full/not active, -1 abort. If `pos_out` is
// given, the position used is stored there.
__device__ int wave_enqueue_one(const Queue& q, bool active, uint32_t val, bool give_up_on_full,
                                unsigned long long limit, unsigned long long& spins,
                                unsigned long long& fails, unsigned long long* pos_out) {
    bool want = active;
    int result = 0;
    int level = 0;
    bq::Watch wd;
    wd.arm(limit);
    while (true) {
        unsigned long long mask = bq::ballot(want);
        if (mask == 0ull) break;
        const uint32_t k = (uint32_t)__popcll(mask);
        const int rank = bq::rank_in(mask);
        uint32_t e = 0;
        unsigned long long base = 0;
        if (bq::lane_id() == 0) {
            e = bq::reserve_enqueue(q, k);
            if (e) base = bq::add_rlx(&q.ctrl->tail.v, (unsigned long long)e);
        }
        e = bq::bcast32(e);
        base = bq::bcast64(base);
        const bool mine = want && rank < (int)e;
        if (e) {
            const unsigned long long pos = base + (unsigned long long)rank;
            if (!bq::put_slots(q, mine, pos, val, limit, spins)) return -1;
            if (mine) {
                result = 1;
                want = false;
                if (pos_out) *pos_out = pos;
            }
        }
        if (bq::ballot(want) == 0ull) break;
        // not ensured: Full (return) or a transient state (retry)
        bool full = false;
        if (bq::lane_id() == 0) full = bq::looks_full(q);
        full = bq::bcast32(full) != 0;
        if (full) {
            if (want) ++fails;
            if (give_up_on_full) break;
        }
        if (bq::aborted(q)) return -1;
        if (wd.expired()) {
            if (bq::lane_id() == 0) bq::raise_error(q, bq::ERR_TIMEOUT);
            return -1;
        }
        bq::backoff(level);
        if (level < 3) ++level;
    }
    return result;
}

// Mirror image for DEQUEUE: returns 1 with `val` set, 0 Empty, -1 abort.
__device__ int wave_dequeue_one(const Queue& q, bool active, uint32_t& val, bool give_up_on_empty,
                                unsigned long long limit, unsigned long long& spins,
                                unsigned long long& fails, unsigned long long* pos_out) {
    bool want = active;
    int result = 0;
    int level = 0;
    bq::Watch wd;
    wd.arm(limit);
    while (true) {
        unsigned long long mask = bq::ballot(want);
        if (mask == 0ull) break;
        const uint32_t k = (uint32_t)__popcll(mask);
        const int rank = bq::rank_in(mask);
        uint32_t e = 0;
        unsigned long long base = 0;
        if (bq::lane_id() == 0) {
            e = bq::reserve_dequeue(q, k);
            if (e) base = bq::add_rlx(&q.ctrl->head.v, (unsigned long long)e);
        }
        e = bq::bcast32(e);
        base = bq::bcast64(base);
        const bool mine = want && rank < (int)e;
        if (e) {
            const unsigned long long pos = base + (unsigned long long)rank;
            uint32_t v = 0;
            if (!bq::read_slots(q, mine, pos, v, limit, spins)) return -1;
            if (mine) {
                val = v;
                result = 1;
                want = false;
                if (pos_out) *pos_out = pos;
            }
        }
        if (bq::ballot(want) == 0ull) break;
        bool empty = false;
        if (bq::lane_id() == 0) empty = bq::looks_empty(q);
        empty = bq::bcast32(empty) != 0;
        if (empty) {
            if (want) ++fails;
            if (give_up_on_empty) break;
        }
        if (bq::aborted(q)) return -1;
        if (wd.expired()) {
            if (bq::lane_id() == 0) bq::raise_error(q, bq::ERR_TIMEOUT);
            return -1;
        }
        bq::backoff(level);
        if (level < 3) ++level;
    }
    return result;
}

__global__ void k_bulk_enqueue(unsigned long long* slots, bq::Ctrl* ctrl, uint32_t logN,
                               const int32_t* vals, unsigned long long n,
                               unsigned long long* n_ok, unsigned long long limit) {
    const Queue q = view(slots, ctrl, logN);
    const unsigned long long waves = (unsigned long long)gridDim.x * (blockDim.x >> 6);
    const unsigned long long wave = (unsigned long long)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    unsigned long long ok = 0, spins = 0, fails = 0;
    for (unsigned long long c = wave; c * 64ull < n; c += waves) {
        const unsigned long long i = c * 64ull + (unsigned long long)bq::lane_id();
        const bool active = i < n;
        const uint32_t v = active ? (uint32_t)vals[i] : 0u;
        int r = wave_enqueue_one(q, active, v, true, limit, spins, fails, nullptr);
        if (__any(r < 0)) break;
        ok += (r == 1);
    }
    // wave reduction of ok
    for (int off = 32; off > 0; off >>= 1) ok += __shfl_xor(ok, off, 64);
    if (bq::lane_id() == 0 && ok) bq::add_rlx(n_ok, ok);
}

__global__ void k_bulk_dequeue(unsigned long long* slots, bq::Ctrl* ctrl, uint32_t logN,
                               int32_t* out, unsigned long long n, unsigned long long* n_ok,
                               unsigned long long limit) {
    const Queue q = view(slots, ctrl, logN);
    const unsigned long long waves = (unsigned long long)gridDim.x * (blockDim.x >> 6);
    const unsigned long long wave = (unsigned long long)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    unsigned long long spins = 0, fails = 0;
    for (unsigned long long c = wave; c * 64ull < n; c += waves) {
        const unsigned long long i = c * 64ull + (unsigned long long)bq::lane_id();
        const bool active = i < n;
        uint32_t v = 0;
        int r = wave_dequeue_one(q, active, v, true, limit, spins, fails, nullptr);
        if (__any(r < 0)) break;
        // compact the successes of this wave, in position order
        const unsigned long long m = bq::ballot(r == 1);
        if (m == 0ull) break;  // queue empty for the whole wave: later waves see it too
        unsigned long long base = 0;
        if (bq::lane_id() == 0) base = bq::add_rlx(n_ok, (unsigned long long)__popcll(m));
        base = bq::bcast64(base);
        if (r == 1) out[base + (unsigned long long)bq::rank_in(m)] = (int32_t)v;
    }
}

// Section IV "Global Mixed": even workgroups enqueue, odd dequeue. A wave
// takes chunks of K = 64*b operations (grid-stride over chunks); each chunk
// is moved with as few broker reservations and head/tail tickets as the
// queue state allows (one of each when it fits), and an attempt that finds
// the queue Full / Empty is retried after a backoff until the chunk is done.
// Enqueue operation i writes value i. stats[0..3] = enq_ok, deq_ok,
// enq_full, deq_empty.
__global__ void k_bench_mixed(unsigned long long* slots, bq::Ctrl* ctrl, uint32_t logN,
                              unsigned long long n_half, int32_t* enq_log, int32_t* deq_log,
                              unsigned long long pos0, unsigned long long* stats,
                              unsigned long long limit, unsigned b) {
    const Queue q = view(slots, ctrl, logN);
    const int lane = bq::lane_id();
    const int wpb = blockDim.x >> 6;
    const bool enq = (blockIdx.x & 1u) == 0u;
    const unsigned long long role_blocks = enq ? (gridDim.x + 1u) / 2u : gridDim.x / 2u;
    const unsigned long long waves = role_blocks * (unsigned long long)wpb;
    const unsigned long long wave = (unsigned long long)(blockIdx.x >> 1) * wpb + (threadIdx.x >> 6);
    const unsigned long long K = 64ull * b;
    unsigned long long ok = 0, spins = 0, fails = 0;
    bool bad = false;
    for (unsigned long long c = wave; c * K < n_half && !bad; c += waves) {
        const unsigned long long first = c * K;
        const unsigned long long cnt = (n_half - first) < K ? (n_half - first) : K;
        unsigned long long done = 0;
        int level = 0;
        bq::Watch wd;
        wd.arm(limit);
        while (done < cnt) {
            uint32_t e = 0;
            unsigned long long base = 0;
            if (lane == 0) {
                const uint32_t want = (uint32_t)(cnt - done);
                e = enq ? bq::reserve_enqueue(q, want) : bq::reserve_dequeue(q, want);
                if (e) base = bq::add_rlx(enq ? &q.ctrl->tail.v : &q.ctrl->head.v,
                                          (unsigned long long)e);
            }
            e = bq::bcast32(e);
            base = bq::bcast64(base);
            for (uint32_t j0 = 0; j0 < e; j0 += 64) {
                const uint32_t j = j0 + (uint32_t)lane;
                const bool act = j < e;
                const unsigned long long pos = base + j;
                if (enq) {
                    const uint32_t val = (uint32_t)(first + done + j);
                    if (!bq::put_slots(q, act, pos, val, limit, spins)) {
                        bad = true;
                        break;
                    }
                    if (act && enq_log) enq_log[pos - pos0] = (int32_t)val;
                } else {
                    uint32_t val = 0;
                    if (!bq::read_slots(q, act, pos, val, limit, spins)) {
                        bad = true;
                        break;
                    }
                    if (act && deq_log) deq_log[pos - pos0] = (int32_t)val;
                }
            }
            if (bad) break;
            done += e;
            ok += e;
            if (done < cnt) {
                ++fails;
                if (bq::aborted(q)) {
                    bad = true;
                    break;
                }
                if (wd.expired()) {
                    if (lane == 0) bq::raise_error(q, bq::ERR_TIMEOUT);
                    bad = true;
                    break;
                }
                bq::backoff(level);
                if (level < 3) ++level;
            }
        }
    }
    if (lane == 0) {
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
        case BQ_EBUSY: return "object too small for this input";
    }
    return "unknown status";
}

int32_t bq_device_cus(void) { return bqh::device_cus(); }

static bq_status queue_zero(bq_queue* q, hipStream_t s) {
    BQ_HIP_TRY(hipMemsetAsync(q->slots, 0, sizeof(unsigned long long) * q->capacity, s));
    BQ_HIP_TRY(hipMemsetAsync(q->ctrl, 0, sizeof(bq::Ctrl), s));
    return BQ_OK;
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
        hipMalloc(&q->ctrl, sizeof(bq::Ctrl)) != hipSuccess ||
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

static bq_status check_error_and_reset(bq_queue* q, hipStream_t s) {
    unsigned long long err = 0;
    BQ_HIP_TRY(hipMemcpyAsync(&err, &q->ctrl->error.v, 8, hipMemcpyDeviceToHost, s));
    BQ_HIP_TRY(hipStreamSynchronize(s));
    if (err != 0ull) {
        queue_zero(q, s);
        BQ_HIP_TRY(hipStreamSynchronize(s));
        return BQ_ETIMEOUT;
    }
    return BQ_OK;
}

static int bulk_grid(const bqh::Launch& L, unsigned long long n) {
    const unsigned long long waves_needed = (n + 63ull) / 64ull;
    const unsigned long long wpb = (unsigned long long)(L.wg_size / 64);
    unsigned long long g = (waves_needed + wpb - 1ull) / wpb;
    if (g > (unsigned long long)L.wg_count) g = (unsigned long long)L.wg_count;
    return g < 1ull ? 1 : (int)g;
}

bq_status bq_enqueue(bq_queue* q, const int32_t* d_vals, uint64_t n, uint64_t* d_n_ok,
                     const bq_launch* launch, void* stream) {
    if (!q || !d_n_ok || (n && !d_vals)) return BQ_EINVAL;
    hipStream_t s = bqh::as_stream(stream);
    bqh::Launch L = bqh::resolve(launch, 4 * bqh::device_cus());
    if (L.wg_size % 64 || L.wg_size > 1024) return BQ_EINVAL;
    BQ_HIP_TRY(hipMemsetAsync(d_n_ok, 0, 8, s));
    if (n) {
        hipLaunchKernelGGL(k_bulk_enqueue, dim3(bulk_grid(L, n)), dim3(L.wg_size), 0, s,
                           q->slots, q->ctrl, q->logN, d_vals, (unsigned long long)n,
                           (unsigned long long*)d_n_ok, L.limit);
        BQ_HIP_TRY(hipGetLastError());
    }
    return check_error_and_reset(q, s);
}

bq_status bq_dequeue(bq_queue* q, int32_t* d_out, uint64_t n, uint64_t* d_n_ok,
                     const bq_launch* launch, void* stream) {
    if (!q || !d_n_ok || (n && !d_out)) return BQ_EINVAL;
    hipStream_t s = bqh::as_stream(stream);
    bqh::Launch L = bqh::resolve(launch, 4 * bqh::device_cus());
    if (L.wg_size % 64 || L.wg_size > 1024) return BQ_EINVAL;
    BQ_HIP_TRY(hipMemsetAsync(d_n_ok, 0, 8, s));
    if (n) {
        hipLaunchKernelGGL(k_bulk_dequeue, dim3(bulk_grid(L, n)), dim3(L.wg_size), 0, s,
                           q->slots, q->ctrl, q->logN, d_out, (unsigned long long)n,
                           (unsigned long long*)d_n_ok, L.limit);
        BQ_HIP_TRY(hipGetLastError());
    }
    return check_error_and_reset(q, s);
}

bq_status bq_bench_mixed(bq_queue* q, uint64_t n_ops, const bq_launch* launch,
                         int32_t* d_enq_log, int32_t* d_deq_log, bq_bench_stats* h_out,
                         int32_t* h_enq_waves, void* stream) {
    if (!q || n_ops < 2 || (n_ops & 1ull) || n_ops / 2 > 0x7fffffffull) return BQ_EINVAL;
    hipStream_t s = bqh::as_stream(stream);
    bqh::Launch L = bqh::resolve(launch, 0);
    if (L.wg_size % 64 || L.wg_size > 1024) return BQ_EINVAL;
    if (L.batch < 1 || 64ull * (unsigned long long)L.batch > q->capacity) return BQ_EINVAL;
    // co-resident grid: enqueuers spin on Full until dequeuers run, so all
    // workgroups must be resident together (cooperative launch checks it)
    int per_cu = 0;
    BQ_HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_bench_mixed, L.wg_size, 0));
    const int max_grid = per_cu * bqh::device_cus();
    int grid = L.wg_count > 0 ? L.wg_count : max_grid;
    if (grid > max_grid) grid = max_grid;
    grid &= ~1;
    if (grid < 2) return BQ_EINVAL;
    // start from an empty, zeroed queue (outside the timed region)
    bq_status st = queue_zero(q, s);
    if (st != BQ_OK) return st;
    BQ_HIP_TRY(hipMemsetAsync(q->scratch, 0, 64, s));
    unsigned long long n_half = n_ops / 2ull;
    unsigned long long pos0 = 0ull;
    int32_t* el = d_enq_log;
    int32_t* dl = d_deq_log;
    unsigned long long* stats = q->scratch;
    unsigned long long* sl = q->slots;
    bq::Ctrl* ct = q->ctrl;
    uint32_t lg = q->logN;
    unsigned long long lim = L.limit;
    unsigned bb = (unsigned)L.batch;
    void* args[] = {&sl, &ct, &lg, &n_half, &el, &dl, &pos0, &stats, &lim, &bb};
    BQ_HIP_TRY(hipEventRecord(q->ev0, s));
    BQ_HIP_TRY(hipLaunchCooperativeKernel((const void*)k_bench_mixed, dim3(grid), dim3(L.wg_size),
                                          args, 0, s));
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
    if (h_enq_waves) *h_enq_waves = ((grid + 1) / 2) * (L.wg_size / 64);
    return st;
}

}  // extern "C"
