// Served form: a request loop over resident graphs and uploaded one-off
// graphs with continuous batching.
//
// - Resident graphs stay in HBM (registered once, device pointers owned by
//   the caller).
// - Per-request device memory (an uploaded graph, engine-owned outputs)
//   comes from one arena allocated at creation; a request is admitted only
//   when its footprint fits what is free, so the hot path never calls
//   hipMalloc.
// - The engine has K lanes, each a stream with its own batched-solver
//   workspace. Whenever a lane is free, it takes the requests that have
//   arrived and fit (in arrival order, up to the lane's batch limits) and
//   starts one batched launch for them; requests that arrive while other
//   launches run are picked up by the next free lane, so their work overlaps
//   on the device. Large requests (enough work for 64 or more workgroups)
//   go alone, so they run with all queue segments and small requests are
//   not held back until a large one in their batch finishes. The last k
//   lanes may be reserved for small requests: a large request at the front
//   of the arrival order holds every lane it can use, and without a reserved
//   lane the small requests behind it wait for it to be launched.
// - Latency = arrival (trace time) to the moment the engine sees the launch
//   complete; the loop runs on the calling thread with a steady clock.
#include <hip/hip_runtime.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <deque>
#include <map>
#include <thread>
#include <vector>

#include "host_common.hpp"

// a request with work for this many workgroups ((n + m/16) / 16K) is large
constexpr long long LARGE_WGS = 64;

#include "arena_host.hpp"

// ---------------------------------------------------------------------------
// the engine
// ---------------------------------------------------------------------------
namespace {

struct ResidentGraph {
    int32_t n;
    int64_t m;
    const int64_t* off;
    const int32_t* col;
    const int32_t* w;
    bool has_launch;   // large requests on this graph use `launch`
    bq_launch launch;
};

struct Lane {
    sssp_batch* batch;
    hipStream_t stream;  // uploads, ordered before the lane's launch
    bool busy;
    std::vector<int> reqs;
    std::vector<uint64_t> blocks;  // arena offsets to free at completion
    std::vector<int32_t> neg;
    std::vector<int64_t> reached;
    double t_launch;
};

uint64_t upload_bytes(int32_t n, int64_t m) {
    return (uint64_t)(n + 1) * 8 + (uint64_t)m * 8 + 1024;
}

}  // namespace

struct bq_server {
    int device;
    int max_batch;
    int small_lanes;  // the last small_lanes lanes take only small requests
    int64_t max_batch_n, max_batch_m;
    bq_launch launch;
    std::vector<Lane> lanes;
    std::vector<ResidentGraph> graphs;
    char* d_arena;
    uint64_t arena_size;
    bq_arena* arena;
};

extern "C" {

bq_status bq_server_destroy(bq_server* s);

bq_status bq_server_create(int32_t lanes, int32_t max_batch, int64_t max_batch_n,
                           int64_t max_batch_m, int64_t arena_bytes, const bq_launch* launch,
                           bq_server** out) {
    if (!out || lanes < 1 || lanes > 16 || max_batch < 1 || max_batch_n < 1 || max_batch_m < 0 ||
        arena_bytes < 4096)
        return BQ_EINVAL;
    *out = nullptr;
    bq_server* s = new bq_server();
    BQ_HIP_TRY(hipGetDevice(&s->device));
    s->max_batch = max_batch;
    s->small_lanes = 0;
    s->max_batch_n = max_batch_n;
    s->max_batch_m = max_batch_m;
    s->launch = launch ? *launch : bq_launch{};
    s->arena_size = (uint64_t)arena_bytes;
    if (hipMalloc(&s->d_arena, s->arena_size) != hipSuccess) {
        delete s;
        return BQ_ENOMEM;
    }
    bq_arena_create(s->arena_size, 256, &s->arena);
    s->lanes.resize(lanes);
    for (auto& L : s->lanes) {
        L.batch = nullptr;
        L.busy = false;
        L.stream = nullptr;
    }
    for (auto& L : s->lanes) {
        bq_status st = sssp_batch_create(max_batch, max_batch_n, max_batch_m, &L.batch);
        if (st != BQ_OK) {
            bq_server_destroy(s);
            return st;
        }
        if (hipStreamCreateWithFlags(&L.stream, hipStreamNonBlocking) != hipSuccess) {
            bq_server_destroy(s);
            return BQ_EHIP;
        }
    }
    *out = s;
    return BQ_OK;
}

bq_status bq_server_destroy(bq_server* s) {
    if (!s) return BQ_OK;
    (void)hipDeviceSynchronize();
    for (auto& L : s->lanes) {
        if (L.batch) sssp_batch_destroy(L.batch);
        if (L.stream) (void)hipStreamDestroy(L.stream);
    }
    if (s->arena) bq_arena_destroy(s->arena);
    if (s->d_arena) (void)hipFree(s->d_arena);
    delete s;
    return BQ_OK;
}

bq_status bq_server_set_small_lanes(bq_server* s, int32_t k) {
    if (!s || k < 0 || k >= (int32_t)s->lanes.size()) return BQ_EINVAL;
    s->small_lanes = k;
    return BQ_OK;
}

bq_status bq_server_add_graph(bq_server* s, int32_t n, int64_t m, const int64_t* d_offsets,
                              const int32_t* d_cols, const int32_t* d_w, int32_t* graph_id) {
    if (!s || !graph_id || n < 1 || m < 0 || !d_offsets || (m > 0 && (!d_cols || !d_w)))
        return BQ_EINVAL;
    if (n > s->max_batch_n || m > s->max_batch_m) return BQ_EBUSY;
    s->graphs.push_back(ResidentGraph{n, m, d_offsets, d_cols, d_w, false, bq_launch{}});
    *graph_id = (int32_t)s->graphs.size() - 1;
    return BQ_OK;
}

bq_status bq_server_set_graph_launch(bq_server* s, int32_t graph_id, const bq_launch* launch) {
    if (!s || graph_id < 0 || graph_id >= (int32_t)s->graphs.size()) return BQ_EINVAL;
    ResidentGraph& g = s->graphs[graph_id];
    g.has_launch = launch != nullptr;
    g.launch = launch ? *launch : bq_launch{};
    return BQ_OK;
}

bq_status bq_server_run(bq_server* s, int32_t count, const bq_request* reqs,
                        bq_response* resp, bq_server_stats* stats) {
    if (!s || count < 0 || (count > 0 && (!reqs || !resp))) return BQ_EINVAL;
    using clk = std::chrono::steady_clock;
    const auto t0 = clk::now();
    auto now_us = [&]() {
        return std::chrono::duration<double, std::micro>(clk::now() - t0).count();
    };
    // a request's size and memory
    struct Need {
        int32_t n;
        int64_t m;
        uint64_t bytes;
    };
    std::vector<Need> need(count);
    for (int i = 0; i < count; ++i) {
        const bq_request& r = reqs[i];
        memset(&resp[i], 0, sizeof(bq_response));
        resp[i].status = BQ_OK;
        resp[i].lane = -1;
        Need nd{0, 0, 0};
        if (r.graph >= 0) {
            if (r.graph >= (int32_t)s->graphs.size()) {
                resp[i].status = BQ_EINVAL;
            } else {
                nd.n = s->graphs[r.graph].n;
                nd.m = s->graphs[r.graph].m;
            }
        } else {
            if (r.n < 1 || r.m < 0 || !r.h_offsets || (r.m > 0 && (!r.h_cols || !r.h_w)))
                resp[i].status = BQ_EINVAL;
            nd.n = r.n;
            nd.m = r.m;
            nd.bytes += upload_bytes(r.n, r.m);
        }
        if (resp[i].status == BQ_OK && (r.src < 0 || r.src >= nd.n)) resp[i].status = BQ_EINVAL;
        if (!r.d_dist) nd.bytes += (uint64_t)nd.n * 12 + 512;
        if (nd.n > s->max_batch_n || nd.m > s->max_batch_m || nd.bytes > s->arena_size)
            resp[i].status = BQ_EBUSY;
        need[i] = nd;
    }
    std::deque<int> pending;
    int next = 0, done = 0;
    uint64_t batches = 0, max_inflight = 0, inflight = 0, max_lanes_busy = 0, upload_total = 0;
    std::vector<sssp_instance> inst;
    inst.reserve(s->max_batch);
    // requests rejected up front complete at their arrival
    while (done < count) {
        const double t = now_us();
        bool progress = false;
        while (next < count && reqs[next].arrival_us <= t) {
            if (resp[next].status != BQ_OK) {
                resp[next].latency_us = 0;
                ++done;
            } else {
                pending.push_back(next);
            }
            ++next;
            progress = true;
        }
        // completions
        int busy_now = 0;
        for (auto& L : s->lanes) {
            if (!L.busy) continue;
            const int k = (int)L.reqs.size();
            bq_status st = sssp_batch_finish(L.batch, L.neg.data(), L.reached.data(), 0);
            if (st == BQ_EBUSY) {
                ++busy_now;
                continue;
            }
            const double tc = now_us();
            for (int j = 0; j < k; ++j) {
                const int i = L.reqs[j];
                resp[i].status = st;
                resp[i].neg_cycle = L.neg[j];
                resp[i].reached_edges = L.reached[j];
                resp[i].latency_us = tc - reqs[i].arrival_us;
                resp[i].service_us = tc - L.t_launch;
            }
            for (uint64_t off : L.blocks) bq_arena_free(s->arena, off);
            L.blocks.clear();
            inflight -= (uint64_t)k;
            done += k;
            L.busy = false;
            L.reqs.clear();
            progress = true;
        }
        // launches: every free lane takes what has arrived and fits
        const std::size_t first_small = s->lanes.size() - (std::size_t)s->small_lanes;
        for (std::size_t li = 0; li < s->lanes.size(); ++li) {
            Lane& L = s->lanes[li];
            const bool small_only = li >= first_small;
            if (L.busy || pending.empty()) continue;
            inst.clear();
            L.reqs.clear();
            L.blocks.clear();
            int64_t sn = 0, sm = 0;
            // size classes: a large request (one that can feed LARGE_WGS or
            // more workgroups on its own) is launched alone, so it runs with the
            // whole queue-segment set and small requests do not wait for it;
            // small requests are batched together in arrival order, passing
            // over large ones, which keep their place at the front; a lane
            // reserved for small requests passes over every large one
            std::size_t scan = 0;
            while (scan < pending.size() && (int)L.reqs.size() < s->max_batch) {
                const int i = pending[scan];
                const Need& nd = need[i];
                const bool large = ((long long)nd.n + nd.m / 16) / 16384 >= LARGE_WGS;
                if (large && (small_only || !L.reqs.empty())) {
                    ++scan;
                    continue;
                }
                if (sn + nd.n > s->max_batch_n || sm + nd.m > s->max_batch_m) break;
                // admission by footprint: uploads and engine-owned outputs
                uint64_t off_up = 0, off_out = 0;
                bool ok = true;
                const bq_request& r = reqs[i];
                const bool up = r.graph < 0;
                if (up && bq_arena_alloc(s->arena, upload_bytes(nd.n, nd.m), &off_up) != BQ_OK)
                    ok = false;
                if (ok && !r.d_dist &&
                    bq_arena_alloc(s->arena, (uint64_t)nd.n * 12 + 512, &off_out) != BQ_OK) {
                    if (up) bq_arena_free(s->arena, off_up);
                    ok = false;
                }
                if (!ok) break;  // arrival order is kept: wait for memory to free up
                pending.erase(pending.begin() + (std::ptrdiff_t)scan);
                sssp_instance q{};
                q.n = nd.n;
                q.m = nd.m;
                q.src = r.src;
                if (up) {
                    char* base = s->d_arena + off_up;
                    int64_t* d_off = (int64_t*)base;
                    int32_t* d_col = (int32_t*)(base + (((uint64_t)(nd.n + 1) * 8 + 255) & ~255ull));
                    int32_t* d_w = d_col + nd.m;
                    if (hipMemcpyAsync(d_off, r.h_offsets, (size_t)(nd.n + 1) * 8,
                                       hipMemcpyHostToDevice, L.stream) != hipSuccess ||
                        (nd.m > 0 &&
                         (hipMemcpyAsync(d_col, r.h_cols, (size_t)nd.m * 4, hipMemcpyHostToDevice,
                                         L.stream) != hipSuccess ||
                          hipMemcpyAsync(d_w, r.h_w, (size_t)nd.m * 4, hipMemcpyHostToDevice,
                                         L.stream) != hipSuccess))) {
                        // this request fails; the lanes and the rest of the
                        // trace go on (its memory is not used by any launch)
                        bq_arena_free(s->arena, off_up);
                        if (!r.d_dist) bq_arena_free(s->arena, off_out);
                        resp[i].status = BQ_EHIP;
                        resp[i].latency_us = now_us() - r.arrival_us;
                        ++done;
                        progress = true;
                        continue;
                    }
                    L.blocks.push_back(off_up);
                    upload_total += upload_bytes(nd.n, nd.m);
                    q.offsets = d_off;
                    q.cols = d_col;
                    q.w = d_w;
                } else {
                    const ResidentGraph& g = s->graphs[r.graph];
                    q.offsets = g.off;
                    q.cols = g.col;
                    q.w = g.w;
                }
                if (r.d_dist) {
                    q.dist = r.d_dist;
                    q.pred = r.d_pred;
                } else {
                    L.blocks.push_back(off_out);
                    q.dist = (int64_t*)(s->d_arena + off_out);
                    q.pred = (int32_t*)(s->d_arena + off_out + (((uint64_t)nd.n * 8 + 255) & ~255ull));
                }
                sn += nd.n;
                sm += nd.m;
                inst.push_back(q);
                L.reqs.push_back(i);
                resp[i].wait_us = now_us() - r.arrival_us;
                if (large) break;
            }
            if (inst.empty()) continue;
            L.neg.assign(inst.size(), 0);
            L.reached.assign(inst.size(), 0);
            bq_launch lo = s->launch;
            // a large request on a resident graph with a launch of its own
            // (launched alone) runs with that launch
            if (inst.size() == 1) {
                const bq_request& r0 = reqs[L.reqs[0]];
                if (r0.graph >= 0 && s->graphs[r0.graph].has_launch &&
                    ((long long)need[L.reqs[0]].n + need[L.reqs[0]].m / 16) / 16384 >= LARGE_WGS)
                    lo = s->graphs[r0.graph].launch;
            }
            bq_status st = sssp_bf_batched_start(L.batch, (int32_t)inst.size(), inst.data(), &lo,
                                                 L.stream);
            if (st != BQ_OK) {
                for (int i : L.reqs) {
                    resp[i].status = st;
                    resp[i].latency_us = now_us() - reqs[i].arrival_us;
                }
                for (uint64_t off : L.blocks) bq_arena_free(s->arena, off);
                done += (int)L.reqs.size();
                L.reqs.clear();
                L.blocks.clear();
                continue;
            }
            for (int i : L.reqs) resp[i].lane = (int32_t)li;
            L.t_launch = now_us();
            L.busy = true;
            ++batches;
            inflight += inst.size();
            if (inflight > max_inflight) max_inflight = inflight;
            progress = true;
        }
        int busy = 0;
        for (auto& L : s->lanes) busy += L.busy ? 1 : 0;
        if ((uint64_t)busy > max_lanes_busy) max_lanes_busy = (uint64_t)busy;
        (void)busy_now;
        if (!progress) {
            // nothing changed: wait a little (or until the next arrival)
            double wait = 20.0;
            if (next < count) {
                const double dt = reqs[next].arrival_us - now_us();
                if (dt < wait) wait = dt > 0 ? dt : 0;
            }
            if (wait > 2.0) std::this_thread::sleep_for(std::chrono::microseconds((long)(wait / 2)));
        }
    }
    if (stats) {
        memset(stats, 0, sizeof *stats);
        stats->wall_ms = now_us() / 1e3;
        stats->launches = batches;
        stats->max_inflight = max_inflight;
        stats->max_lanes_busy = max_lanes_busy;
        uint64_t used = 0, peak = 0;
        bq_arena_usage(s->arena, &used, &peak, nullptr);
        stats->arena_peak_bytes = peak;
        stats->upload_bytes = upload_total;
    }
    return BQ_OK;
}

}  // extern "C"
