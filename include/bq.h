/*
 * bq.h - C ABI of the MI355X Broker-Queue / queue-driven Bellman-Ford library
 * (libbqsssp.so, built for gfx950).
 *
 * Two groups of entry points:
 *
 *  1. The concurrent FIFO of Section III.A (Alg. 1, the Broker Queue):
 *     bq_create / bq_destroy / bq_reset (INITIALIZE), bq_enqueue (ENQUEUE,
 *     Successful or Full), bq_dequeue (DEQUEUE, data or Empty) and
 *     bq_bench_mixed (the "Global Mixed" scenario of Section IV: even
 *     workgroups enqueue, odd workgroups dequeue, concurrently).
 *
 *  2. Single-source shortest paths with the queue-based Bellman-Ford of
 *     Section III.C, whose input and output are those of Alg. 3 (graph G,
 *     source s -> distances d and the negative-cycle detection):
 *     sssp_ctx_create / sssp_ctx_destroy, sssp_bf (one query) and
 *     sssp_batch_create / sssp_bf_batched (many queries in one persistent
 *     launch).
 *
 * Conventions for every call:
 *  - Pointers named d_* are device pointers (HBM of the current HIP device),
 *    h_* are host pointers. The caller owns every buffer it passes; the
 *    library keeps no caller pointer after the call returns.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *  - Every call returns a bq_status; outputs are unspecified unless BQ_OK.
 *    A NULL handle gives BQ_EINVAL before any HIP call, except in the
 *    *_destroy calls, which accept NULL and return BQ_OK.
 *  - Integer arithmetic only: int32 weights, int64 distances.
 *  - The library never allocates on a solve: queues and workspaces are
 *    allocated by bq_create / sssp_ctx_create and reused.
 *  - Calls on one bq_queue or one sssp_ctx must not overlap in time
 *    (they share its device state); distinct objects are independent.
 */
#ifndef BQ_H
#define BQ_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    BQ_OK = 0,
    BQ_EINVAL = -1,   /* bad argument: null pointer, size, malformed CSR */
    BQ_ENOMEM = -2,   /* device or pinned allocation failed */
    BQ_EHIP = -3,     /* a HIP runtime call failed */
    BQ_ERANGE = -4,   /* distances cannot be packed: n * max|w| too large */
    BQ_ETIMEOUT = -5, /* a device-side watchdog fired; state was reset */
    BQ_EBUSY = -6,    /* object too small for this input (max_n / max_m) */
    BQ_EOVERFLOW = -7 /* a solver queue was found over capacity: the queues are
                         sized so that this cannot happen, so it reports a
                         library fault; the state is rebuilt on the next call */
} bq_status;

/* Opaque handles. */
typedef struct bq_queue bq_queue;
typedef struct sssp_ctx sssp_ctx;
typedef struct sssp_batch sssp_batch;
typedef struct sssp_rounds_ctx sssp_rounds_ctx;

/* Launch shape. Zero fields mean "library default". */
typedef struct {
    int32_t wg_size;      /* threads per workgroup, multiple of 64 (<= 1024) */
    int32_t wg_count;     /* workgroups; 0 = the call's default: queue
                             benchmarks fill the chip (occupancy x CUs);
                             sssp_bf and sssp_bf_batched take about one per
                             16K units of n + m/16 (per query, at least one),
                             up to the co-resident maximum */
    int32_t ticket_batch; /* b: a wave dequeues up to 64*b items per ticket;
                             0 = 1; the solvers take 1, 2 or 4 (BQ_EINVAL
                             otherwise: their LDS staging grows with b) */
    uint32_t flags;       /* BQ_F_* */
    uint64_t timeout_us;  /* watchdog for a single wait; 0 = 2 s. A solve
                             running longer than 10x this is stopped too
                             (BQ_ETIMEOUT), so no launch runs unbounded. */
    int32_t row_chunk;    /* solver: rows longer than this many edges are split
                             into queue items of this size (power of two,
                             64..65536); 0 = 128 for sssp_bf, 1024 for
                             the batched form */
    int32_t queue_scale;  /* batched solver: each query's queue holds
                             pow2(queue_scale * (n + m/row_chunk + 1)) slots,
                             1 or 2; 0 = 2 */
    int32_t segments;     /* sssp_bf: the queue is split into this many
                             Broker Queues (1..8, one per XCD), workgroup i
                             publishing to segment i mod segments and taking
                             from the fullest other segment when its own is
                             empty; 0 = min(8, workgroups). Forced to 1 with
                             BQ_F_TRACE. bq_bench_mixed / bq_bench_enqdeq:
                             1, 2, 4 or 8 segments of capacity/segments
                             slots (0 = 1). Other calls ignore it. */
    int32_t bucket_width; /* sssp_bf, sssp_bf_noalloc: 0 = every home segment
                             keeps one FIFO of improved vertices (the method as
                             the paper runs it); k > 0 = near / far buckets: a
                             vertex whose new label is at or above a threshold
                             T goes to a far queue that waves take only when
                             no near work is queued, and a far batch moves T
                             to its smallest label + k * max(1, max |w|) / 16
                             (at least 1).
                             Same results, fewer relabels on large-diameter
                             graphs; the autotuner tries it. Needs one more
                             queue per segment. Other calls ignore it. */
} bq_launch;

#define BQ_F_VALIDATE 1u  /* sssp_bf: check the CSR on the device first */
#define BQ_F_TRACE 2u     /* sssp_bf: record a timeline (see sssp_last_trace) */
#define BQ_F_BWD 8u       /* the Broker Work Distributor policy (Section III.A):
                             single-shot broker check. Queue operations: an
                             operation whose reservation falls short returns
                             Full / Empty at once instead of re-checking head
                             and tail. sssp_bf / sssp_bf_batched: each dequeue
                             takes from the count once, with no look before
                             or after. Results are the same under both. */
#define BQ_F_NEGINF 16u   /* sssp_bf, sssp_bf_batched, sssp_bf_rounds: a negative
                             cycle does not stop the solve; the vertices it
                             makes unbounded are marked instead: dist[v] =
                             INT64_MIN for every v reachable from a negative
                             cycle that src reaches (pred[v] = -1), exact
                             distances and predecessors for the others, and
                             the negative-cycle flag is still set. */
#define BQ_F_NOREMAP 32u  /* sssp_bf_batched: keep the keys of queries that share a
                             graph in vertex order in their dist buffers. By
                             default each graph that two or more queries of the
                             batch share gets a degree-class key layout in the
                             workspace (key positions ordered by out-degree
                             class, highest first, then by id), rebuilt on
                             every call; results are the same bytes either way */
#define BQ_F_GRAPH 4u     /* sssp_bf_batched: run the launch sequence as a hipGraph,
                             captured on first use and replayed while the batch
                             keeps its count and shape */

/* Counters of one bq_bench_mixed run. */
typedef struct {
    uint64_t enq_ok, deq_ok;      /* successful operations */
    uint64_t enq_full, deq_empty; /* attempts that returned Full / Empty and were retried */
    double ms;                    /* kernel time (HIP events) */
} bq_bench_stats;

/* Work counters of the last sssp_bf / sssp_bf_batched call on a context. */
typedef struct {
    uint64_t dequeued;     /* items taken from the queue */
    uint64_t relaxations;  /* edges scanned */
    uint64_t pushes;       /* vertices enqueued after an improvement */
    uint64_t fanout;       /* row chunks of high-degree vertices enqueued */
    uint64_t batches;      /* wave dequeue batches */
    uint64_t walks;        /* parent-pointer walks (negative-cycle search) */
    uint64_t improvements; /* successful atomicMin lowering a distance */
    uint64_t idle_polls;   /* dequeue attempts that found the queue empty */
    uint64_t ticket_spins; /* extra polls of slot words in ticket waits */
    double ms;             /* device time of the call (HIP events) */
    double solve_ms;       /* the persistent solver kernel alone (HIP events) */
    int32_t grid;          /* workgroups launched */
    int32_t wg_size;
} sssp_stats;

/* Counters of the last sssp_bf_rounds call. */
typedef struct {
    uint64_t rounds;       /* rounds run; the last saw no change unless a
                              negative cycle or an error ended the solve */
    uint64_t changes;      /* relaxations that lowered a distance, all rounds */
    uint64_t relaxations;  /* rounds * m: every round relaxes every edge */
    uint64_t ticket_spins; /* extra polls of slot words in ticket waits */
    double ms;             /* device time of the call (HIP events) */
    double solve_ms;       /* the rounds alone (HIP events) */
    int32_t grid;          /* workgroups per round kernel */
    int32_t wg_size;
} sssp_rounds_stats;

/* One query of sssp_bf_batched: all pointers are device pointers (the
 * layouts and outputs of sssp_bf). */
typedef struct {
    int32_t n;               /* vertices */
    int32_t src;             /* source vertex */
    int64_t m;               /* edges */
    const int64_t* offsets;  /* [n+1] CSR row offsets, offsets[0] = 0, offsets[n] = m */
    const int32_t* cols;     /* [m] edge targets */
    const int32_t* w;        /* [m] edge weights */
    int64_t* dist;           /* [n] out */
    int32_t* pred;           /* [n] out, may be NULL */
} sssp_instance;

/* ------------------------------------------------------------------------
 * Queue (Section III.A, Alg. 1)
 * ------------------------------------------------------------------------ */

/* INITIALIZE: allocate a queue of `capacity` int32 slots (a power of two,
 * >= 64) with head = tail = count = 0 and all tickets 0.
 * `flags` is reserved (pass 0). Returns BQ_EINVAL for a bad capacity,
 * BQ_ENOMEM if the device allocation fails. */
bq_status bq_create(uint32_t capacity, uint32_t flags, void* stream, bq_queue** out);

/* Free the queue (synchronizes the device first). NULL is accepted. */
bq_status bq_destroy(bq_queue* q);

/* INITIALIZE again on `stream` (head = tail = count = 0, tickets and slots
 * zeroed). Needed after BQ_ETIMEOUT. */
bq_status bq_reset(bq_queue* q, void* stream);

/* ENQUEUE of n values d_vals[0..n) by a launch of wave-aggregated lanes (a
 * wave moves chunks of 64*b values, b = launch->ticket_batch, 64*b <=
 * capacity; BQ_F_BWD selects the single-shot broker check).
 * Each value is Successful or Full (Alg. 1); with no concurrent dequeuer the
 * first min(n, capacity - size) positions taken succeed. *d_n_ok (device,
 * uint64, overwritten) receives the number of successes. Which values
 * succeed, and their order in the queue, depend on the schedule, except for
 * launch->wg_count = 1 and wg_size = 64 (one wave), which enqueues in array
 * order. launch may be NULL. n = 0 launches nothing and writes 0 to *d_n_ok
 * (d_vals may then be NULL). BQ_EINVAL for a NULL queue or d_n_ok, a NULL
 * d_vals with n > 0, or a launch shape the queue cannot take.
 * Synchronous (returns after completion). */
bq_status bq_enqueue(bq_queue* q, const int32_t* d_vals, uint64_t n, uint64_t* d_n_ok,
                     const bq_launch* launch, void* stream);

/* DEQUEUE up to n values into d_out[0..*d_n_ok) (compacted; Empty for the
 * rest). With one wave (see bq_enqueue) the values come out in queue order.
 * Arguments and n = 0 as for bq_enqueue (d_out may be NULL when n = 0).
 * Synchronous. */
bq_status bq_dequeue(bq_queue* q, int32_t* d_out, uint64_t n, uint64_t* d_n_ok,
                     const bq_launch* launch, void* stream);

/* Section IV "Global Enqueue-Dequeue" (EnqDeq): n_ops/2 enqueues (value i
 * for operation i), then n_ops/2 dequeues, each operation one attempt
 * (Successful / Full, data / Empty), chunks of 64*b per wave as in
 * bq_enqueue. The queue is reset to empty first. *h_enq / *h_deq get the
 * counts and kernel times of the two phases. launch->segments S = 2, 4, 8
 * selects the partitioned form of bq_bench_mixed (segment s carries
 * operations [s P, (s+1) P), P = n_ops/2 / S). Synchronous. */
bq_status bq_bench_enqdeq(bq_queue* q, uint64_t n_ops, const bq_launch* launch,
                          bq_bench_stats* h_enq, bq_bench_stats* h_deq, void* stream);

/* Host view of the queue counters (synchronizes the stream). */
bq_status bq_counters(bq_queue* q, void* stream, uint64_t* h_head, uint64_t* h_tail,
                      int64_t* h_count);

/* Section IV "Global Mixed": a co-resident grid in which even workgroups
 * perform n_ops/2 enqueues and odd workgroups n_ops/2 dequeues. A wave takes
 * chunks of K = 64*b operations (b = launch->ticket_batch, 64*b <= capacity)
 * and moves each chunk with one broker reservation and one head/tail ticket
 * when the queue state allows; attempts that find the queue Full / Empty are
 * counted and retried until every operation succeeded. The queue is reset to
 * empty first. The value enqueued by operation i is i. If d_enq_log /
 * d_deq_log are not NULL (device, int32[n_ops/2] each) the value written at /
 * read from queue position P is stored at index P, for checking the
 * position rule, conservation and per-producer order (launch->flags may
 * select BQ_F_BWD): value i belongs to
 * chunk c = i / K of enqueuer wave c mod W (W = *h_enq_waves on return),
 * lane (i mod K) mod 64 of that wave, and is that lane's item number
 * (c / W) * b + (i mod K) / 64. Synchronous.
 *
 * Partitioned form (launch->segments S = 2, 4 or 8; the paper's multi-GPU
 * queue of Alg. 2 on the chip's XCDs): the queue is split into S Broker
 * Queues of capacity/S slots each (at least 64*b), workgroup i works on
 * segment i mod S and enqueues when (i / S) is even; segment s carries
 * operations [s P, (s+1) P) of each kind, P = n_ops/2 / S (n_ops/2 must be
 * a multiple of S), and the grid is rounded down to a multiple of 2S. Each
 * segment is FIFO on its own. The logs hold position p of segment s at index
 * s P + p; the rule for value i above applies within its segment with
 * i - s P for i, c = (i - s P) / K and W / S enqueuer waves per segment. */
bq_status bq_bench_mixed(bq_queue* q, uint64_t n_ops, const bq_launch* launch,
                         int32_t* d_enq_log, int32_t* d_deq_log, bq_bench_stats* h_out,
                         int32_t* h_enq_waves, void* stream);

/* ------------------------------------------------------------------------
 * Queue-based Bellman-Ford SSSP (Section III.C; Alg. 3's inputs/outputs)
 * ------------------------------------------------------------------------ */

/* Workspace for graphs with n <= max_n and m <= max_m: the vertex queue,
 * control block and chunk table. Allocated once; calls reuse it. */
bq_status sssp_ctx_create(int32_t max_n, int64_t max_m, sssp_ctx** out);
bq_status sssp_ctx_destroy(sssp_ctx* ctx);

/* Single-source shortest paths from src over the CSR graph
 * (d_offsets int64[n+1], d_cols int32[m], d_w int32[m]).
 *
 * Output: d_dist int64[n]: the exact shortest distance, INT64_MAX for
 * vertices not reachable from src (the paper's infinity);
 * d_pred int32[n] (may be NULL): the smallest-id in-neighbour u with
 * dist[u] + w(u,v) == dist[v], -1 for src and unreachable vertices;
 * *h_neg_cycle: 1 if a negative cycle is reachable from src (then dist and
 * pred are unspecified, unless BQ_F_NEGINF is set: see the flag), else 0.
 * A negative cycle is a result, not an error.
 *
 * Self-loops and parallel edges are allowed. Requires 1 <= n <= max_n,
 * 0 <= m <= max_m, 0 <= src < n; with BQ_F_VALIDATE the CSR itself is
 * checked (BQ_EINVAL). BQ_ERANGE when n * max|w| does not fit the packed
 * 64-bit key (bits for the distance = 62 - ceil(log2(n+1))).
 * Synchronous: returns when the outputs are final. launch may be NULL. */
bq_status sssp_bf(sssp_ctx* ctx, int32_t n, int64_t m, const int64_t* d_offsets,
                  const int32_t* d_cols, const int32_t* d_w, int32_t src, int64_t* d_dist,
                  int32_t* d_pred, int32_t* h_neg_cycle, const bq_launch* launch,
                  void* stream);

/* sssp_bf without a context, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc). Same arguments, outputs, conventions and errors as
 * sssp_bf minus the context; it calls no allocating routine. Its workspace
 * (queue slots, control blocks, chunk table) lives in a device array of
 * 128 MiB that the library's code object reserves on every device it runs
 * on, for the life of the process; each call clears the part it uses.
 * Limit: with S queue segments (launch->segments, default min(8,
 * workgroups)), 2 S P slots of 8 bytes, P = the power of two >= 2 (n +
 * m/64 + 1) and >= 4096, plus about 100 KiB + 4 m / C bytes (C = row
 * chunk) must fit 128 MiB: n + m/64 + 1 <= 2^18 with 8 segments, <= 2^21
 * with one (an ER graph of 200k vertices and 1.6M edges fits with 8).
 * Larger inputs return BQ_EBUSY. BQ_F_TRACE
 * is rejected (BQ_EINVAL). All calls on one device share the array: calls
 * that overlap in time on one device race and give undefined results.
 * Synchronous. */
bq_status sssp_bf_noalloc(int32_t n, int64_t m, const int64_t* d_offsets, const int32_t* d_cols,
                          const int32_t* d_w, int32_t src, int64_t* d_dist, int32_t* d_pred,
                          int32_t* h_neg_cycle, const bq_launch* launch, void* stream);

/* Autotuner: time sssp_bf on this input (d_dist is used as scratch). Unless
 * base->bucket_width is set, a few runs at the default grid with and without
 * near / far buckets first pick the order of work (buckets when they are at
 * least 20 % faster); then, in that family: workgroup counts 4, 8, 16, ...
 * up to the co-resident maximum (stopping
 * once clearly past the fastest) and 3/4 and 3/2 of the fastest, then
 * ticket batches b = 2, 4 around the
 * fastest count, then row chunks 64 and 256 at the fastest shape, then
 * 1, 2 and 4 queue segments against the default, and with buckets bucket
 * widths 1, 2 and 16 against the family's 4 (steps of 1/16, 1/8, 1 and 1/4
 * of max |w|); `reps` runs per candidate
 * (0 = 5), compared by their median, a candidate replacing the fastest so
 * far only when at least 3 % faster; a winner that differs from the best
 * power-of-two count with default settings is finally run against it,
 * 2 * reps times each, alternating, and kept only if its median is lower.
 * *h_best gets the fastest launch (other fields copied from `base`, which
 * may be NULL), *h_best_ms its time. Synchronous. */
bq_status sssp_autotune(sssp_ctx* ctx, int32_t n, int64_t m, const int64_t* d_offsets,
                        const int32_t* d_cols, const int32_t* d_w, int32_t src, int64_t* d_dist,
                        const bq_launch* base, int32_t reps, bq_launch* h_best,
                        double* h_best_ms, void* stream);

/* Work counters and device time of the last call on ctx. */
bq_status sssp_last_stats(const sssp_ctx* ctx, sssp_stats* h_out);

/* Timeline of the last sssp_bf call made with BQ_F_TRACE (one vertex queue):
 * up to cap_samples samples of 4 uint64 each, (time since start in 10 ns
 * ticks, vertex items dequeued so far, vertex queue length, pending work
 * including the waves' unpaid debts); one sample each time the dequeued
 * vertex items cross a multiple of 2^k (k chosen from n and m), unused
 * samples all ones. Returns the number of samples written, or BQ_EINVAL. */
int32_t sssp_last_trace(const sssp_ctx* ctx, uint64_t* h_out, int32_t cap_samples);

/* ------------------------------------------------------------------------
 * Round-based Bellman-Ford over an edge queue (Section III.C's single-GPU
 * form; Alg. 3 on one processing element)
 * ------------------------------------------------------------------------ */

/* Workspace for graphs with n <= max_n and m <= max_m: an edge queue of
 * pow2(max_m) slots (at least 4096; 8 bytes each), the edge-source array
 * (4 bytes per edge) and the control block. BQ_EINVAL if max_m > 2^31. */
bq_status sssp_rounds_create(int32_t max_n, int64_t max_m, sssp_rounds_ctx** out);
bq_status sssp_rounds_destroy(sssp_rounds_ctx* ctx);

/* The paper's own form of the method: the Broker Queue holds edges. Round i
 * (i = 0 .. n-1) enqueues every edge id and the same launch dequeues and
 * relaxes them concurrently (d[v] = min(d[v], d[u] + w) when d[u] is
 * finite, by atomicMin), counting the lowered distances; a round with no
 * change ends the solve, a change in round n-1 proves a negative cycle.
 * So the work is (rounds run) * m relaxations, up to n * m.
 *
 * Inputs, outputs, conventions and errors are those of sssp_bf (same CSR
 * arrays, dist INT64_MAX when unreached, pred = smallest-id tight
 * in-neighbour, -1 for src and unreached; *h_neg_cycle = 1 leaves dist and
 * pred unspecified unless BQ_F_NEGINF is set), except:
 *  - BQ_ERANGE when (n+1) * (m+1) * max|w| >= 2^62 (the distances after n
 *    rounds must not overflow int64);
 *  - launch: wg_size 64..1024 (power of two), wg_count 0 = 2 per CU
 *    (clamped to the co-resident maximum), ticket_batch b = 1..64 edge ids
 *    per lane per queue operation (0 = 16), BQ_F_BWD and BQ_F_VALIDATE as
 *    for sssp_bf, and BQ_F_NEGINF (minus-infinity marking, see the flag);
 *    row_chunk, queue_scale and segments are ignored;
 *  - BQ_ETIMEOUT when one wait exceeds timeout_us or the whole solve
 *    exceeds 10 x timeout_us (checked between groups of rounds).
 * Synchronous. */
bq_status sssp_bf_rounds(sssp_rounds_ctx* ctx, int32_t n, int64_t m, const int64_t* d_offsets,
                         const int32_t* d_cols, const int32_t* d_w, int32_t src,
                         int64_t* d_dist, int32_t* d_pred, int32_t* h_neg_cycle,
                         const bq_launch* launch, void* stream);

/* Counters and device time of the last sssp_bf_rounds call on ctx. */
bq_status sssp_rounds_last_stats(const sssp_rounds_ctx* ctx, sssp_rounds_stats* h_out);

/* ------------------------------------------------------------------------
 * Roofline probes (measurement only)
 * ------------------------------------------------------------------------ */

/* Time one probe kernel with HIP events on `stream` (synchronous):
 *  kind 0: stream copy of `size` bytes (multiple of 16) from d_a to d_b -
 *          the HBM bandwidth probe and the calibration kernel for byte
 *          counters;
 *  kind 1: grid*block lanes each do ops_per_lane (multiple of 4) returning
 *          64-bit atomicMin at random slots of the int64 table d_a of `size`
 *          words (power of two); d_b: 8 bytes of scratch;
 *  kind 2: grid*block lanes each do ops_per_lane atomicAdd on the single
 *          uint64 d_a[0] (16 bytes needed);
 *  kind 3: like kind 2 but one lane per wave (the leader-lane pattern);
 *  kind 4: one lane per wave, ops_per_lane agent-scope loads of d_a[0];
 *  kind 5: grid*block lanes each do ops_per_lane (multiple of 8)
 *          agent-scope 64-bit loads at random words of the table d_a of
 *          `size` words (power of two), 8 in flight; d_b: 8 bytes of scratch;
 *  kind 6 / 7: latency: every lane runs a dependent chain of ops_per_lane
 *          agent-scope loads (6) or returning atomicMins that leave the
 *          word unchanged (7) at random words of the table d_a of `size`
 *          words (power of two); d_b: 8 bytes of scratch;
 *  kind 8: the wave primitives the kernels use, on the int32 d_a[size]
 *          (size = grid * block, block a multiple of 64): per input i,
 *          d_b[4i .. 4i+3] = inclusive sum scan, inclusive unsigned max scan,
 *          the value of the lane below (0 for lane 0) and the value of lane
 *          63, each over the input's wave of 64.
 * *h_ms receives the kernel time. */
bq_status bq_probe(int32_t kind, void* d_a, void* d_b, uint64_t size, uint64_t ops_per_lane,
                   int32_t grid, int32_t block, double* h_ms, void* stream);

/* ------------------------------------------------------------------------
 * Batched form: many queries in one persistent launch
 * ------------------------------------------------------------------------ */

/* Workspace for batches of at most max_instances queries whose vertex and
 * edge counts sum to at most max_total_n / max_total_m: one Broker Queue per
 * query (slots + control block), chunk tables, the query table. */
bq_status sssp_batch_create(int32_t max_instances, int64_t max_total_n, int64_t max_total_m,
                            sssp_batch** out);
bq_status sssp_batch_destroy(sssp_batch* b);

/* Solve `count` independent queries (each its own CSR graph, source and
 * outputs, all device pointers; graphs may be shared between queries) in one
 * launch: every query gets the result sssp_bf would give it alone (dist,
 * pred, h_neg_cycle[i]). Queries are ordered by size; persistent workgroups
 * claim them biggest first, each query getting workgroups in proportion to
 * its edges + vertices, and workgroups whose claims are used up join
 * unfinished queries. Claims come from one list per XCD (workgroup i takes
 * from list i mod 8): a query whose share fits one XCD's workgroups is
 * listed on one list only and keeps one queue segment; a bigger query is
 * spread over all lists, and one with (n + m/16) / 16384 >= 16 gets up to 8
 * queue segments (as sssp_bf) while the workspace's slots allow, biggest
 * first. With BQ_F_GRAPH the init / solve / unpack kernels run
 * as one replayed hipGraph on the batch's own stream (ordered after the
 * caller's stream). Synchronous. Errors: BQ_EINVAL (a bad query), BQ_EBUSY
 * (batch larger than the workspace), BQ_ERANGE / BQ_ETIMEOUT (first failing
 * query; others still have their results). */
bq_status sssp_bf_batched(sssp_batch* b, int32_t count, const sssp_instance* h_inst,
                          int32_t* h_neg_cycle, const bq_launch* launch, void* stream);

/* The two halves of sssp_bf_batched, for callers that overlap work: _start
 * queues the launch (after work already queued on `stream`) and returns at
 * once; sssp_batch_finish collects it: with wait = 0 it returns BQ_EBUSY
 * while the launch runs. h_reached_edges (may be NULL) receives, per query,
 * the number of edges whose source vertex was reached. A batch object runs
 * one launch at a time (BQ_EBUSY from _start otherwise). */
bq_status sssp_bf_batched_start(sssp_batch* b, int32_t count, const sssp_instance* h_inst,
                                const bq_launch* launch, void* stream);
bq_status sssp_batch_finish(sssp_batch* b, int32_t* h_neg_cycle, int64_t* h_reached_edges,
                            int32_t wait);

/* Work counters (summed over the batch) and device time of the last call. */
bq_status sssp_batch_last_stats(const sssp_batch* b, sssp_stats* h_out);

/* Autotuner for a batch: workgroup counts 16, 32, ... up to the co-resident
 * maximum, then row chunks 256 / 4096, ticket batches 2 and 4 and
 * queue_scale 1 at the fastest shape; `reps` runs per candidate (0 = 3)
 * compared by their median, a candidate replacing the fastest so far only
 * when at least 3 % faster. Returns the fastest launch and its time. The
 * result is kept per shape bucket (powers of two of the query count, total
 * vertices and total edges, and base->flags): a later call on the same
 * batch workspace with a batch of the same bucket returns it at once. */
bq_status sssp_batch_autotune(sssp_batch* b, int32_t count, const sssp_instance* h_inst,
                              const bq_launch* base, int32_t reps, bq_launch* h_best,
                              double* h_best_ms, void* stream);

/* ------------------------------------------------------------------------
 * Served form: resident graphs, admission by memory, continuous batching
 * ------------------------------------------------------------------------ */

typedef struct bq_server bq_server;

/* One request of a replayed trace. */
typedef struct {
    double arrival_us;        /* arrival time, microseconds after the run starts;
                                 requests must be sorted by it */
    int32_t graph;            /* resident graph id, or -1: upload the host CSR below */
    int32_t src;
    int32_t n;                /* upload only: host CSR (pinned memory keeps the copy */
    int64_t m;                /*   asynchronous) */
    const int64_t* h_offsets;
    const int32_t* h_cols;
    const int32_t* h_w;
    int64_t* d_dist;          /* device outputs, may be NULL (then the engine uses */
    int32_t* d_pred;          /*   its own memory and the result is dropped) */
} bq_request;

typedef struct {
    double latency_us;        /* arrival -> completion seen by the engine */
    double wait_us;           /* arrival -> its launch was queued */
    double service_us;        /* launch queued -> completion */
    int64_t reached_edges;    /* edges whose source vertex was reached */
    int32_t neg_cycle;
    int32_t status;           /* bq_status of the request: BQ_EINVAL / BQ_EBUSY if
                                 rejected, BQ_EHIP if its upload failed, else the
                                 status of its batched launch */
    int32_t lane;             /* lane whose launch ran it, -1 if it never ran */
    int32_t reserved_;
} bq_response;

typedef struct {
    double wall_ms;
    uint64_t launches;        /* batched launches started */
    uint64_t max_inflight;    /* most requests on the device at once */
    uint64_t max_lanes_busy;  /* most concurrent launches */
    uint64_t arena_peak_bytes;
    uint64_t upload_bytes;
} bq_server_stats;

/* An engine with `lanes` streams (1..16), each able to run one batched
 * launch of up to max_batch requests whose vertex / edge counts sum to at
 * most max_batch_n / max_batch_m, and an arena of arena_bytes of device
 * memory for per-request data (uploaded graphs, engine-owned outputs).
 * `launch` (may be NULL) is the launch shape of every batched launch. */
bq_status bq_server_create(int32_t lanes, int32_t max_batch, int64_t max_batch_n,
                           int64_t max_batch_m, int64_t arena_bytes, const bq_launch* launch,
                           bq_server** out);
bq_status bq_server_destroy(bq_server* s);

/* Reserve the last k lanes (0 <= k < lanes; 0 at creation) for small
 * requests, those with work for fewer than 64 workgroups
 * ((n + m/16) / 16384 < 64). A large request is launched alone on one of the
 * other lanes and, at the front of the arrival order, holds those lanes to
 * itself; a reserved lane passes over it, so small requests that arrive
 * behind large ones still start as soon as a reserved lane is free. The
 * price: large requests have k lanes fewer. BQ_EINVAL for k out of range;
 * no device work. */
bq_status bq_server_set_small_lanes(bq_server* s, int32_t k);

/* Register a resident graph (device CSR owned by the caller, kept valid
 * while the server lives); returns its id. */
bq_status bq_server_add_graph(bq_server* s, int32_t n, int64_t m, const int64_t* d_offsets,
                              const int32_t* d_cols, const int32_t* d_w, int32_t* graph_id);

/* Give the large requests on resident graph graph_id (those launched alone:
 * work for 64 or more workgroups, (n + m/16) / 16384 >= 64) a launch of their
 * own instead of the server's, e.g. one found by sssp_autotune for that graph
 * (near / far buckets for a road mesh). NULL restores the server's launch.
 * BQ_EINVAL for an unknown graph id; no device work. */
bq_status bq_server_set_graph_launch(bq_server* s, int32_t graph_id, const bq_launch* launch);

/* Replay `count` requests at their arrival times on the calling thread:
 * arrived requests wait in arrival order; a request is admitted when its
 * memory (upload + engine outputs) fits the free arena and its sizes fit the
 * free lane's limits; every free lane starts one batched launch with what is
 * admitted, so requests arriving while others run are launched on other
 * lanes and overlap with them. Fills resp[i] per request and *stats
 * (may be NULL). Returns when every request is done; a failing request
 * (rejected, upload or launch error) ends with its own status and does not
 * stop the others. */
bq_status bq_server_run(bq_server* s, int32_t count, const bq_request* reqs,
                        bq_response* resp, bq_server_stats* stats);

/* The engine's first-fit memory arena as a pure host allocator over offsets
 * (exported so the admission logic can be tested without a device).
 * Allocation sizes are rounded up to `align` (a power of two); alloc
 * returns BQ_EBUSY when no free block is large enough; free coalesces. */
typedef struct bq_arena bq_arena;
bq_status bq_arena_create(uint64_t size, uint64_t align, bq_arena** out);
bq_status bq_arena_destroy(bq_arena* a);
bq_status bq_arena_alloc(bq_arena* a, uint64_t bytes, uint64_t* offset);
bq_status bq_arena_free(bq_arena* a, uint64_t offset);
bq_status bq_arena_usage(const bq_arena* a, uint64_t* used, uint64_t* peak,
                         uint64_t* largest_free);

/* Text for a status code (static storage). */
const char* bq_strerror(bq_status s);

/* Number of compute units of the current device (for launch sizing). */
int32_t bq_device_cus(void);

#ifdef __cplusplus
}
#endif
#endif /* BQ_H */
