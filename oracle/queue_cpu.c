/*
 * CPU models of the queue for the benchmark's CPU baselines (test and
 * measurement infrastructure only, like the rest of this directory; the
 * HIP library shares nothing with it).
 *
 *  - cpu_ring_mixed: a sequential bounded ring on one core running the
 *    "Global Mixed" operation sequence (enqueue, dequeue, enqueue, ...), the
 *    single-thread reference point.
 *  - cpu_bq_mixed: the Broker Queue of Section III.A (Alg. 1) with C11
 *    atomics on host threads, one operation per call as the paper writes
 *    it: ENSURE on the broker count (re-checked while the count allows),
 *    a position from head / tail, and the per-slot ticket handshake
 *    (enqueuer of round r waits for ticket 2r, writes, sets 2r+1; dequeuer
 *    waits for 2r+1, reads, sets 2(r+1)). Half the threads enqueue, half
 *    dequeue; an operation that finds the queue Full / Empty is retried, so
 *    every operation completes. Optional logs record the value at each
 *    position for the history checks.
 */
#include <pthread.h>
#include <sched.h>
#include <stdatomic.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

static double now_s(void)
{
    struct timespec t;
    clock_gettime(CLOCK_MONOTONIC, &t);
    return (double)t.tv_sec + 1e-9 * (double)t.tv_nsec;
}

/* Sequential ring: n_ops operations alternating enqueue / dequeue on a ring
 * of cap slots (never Full or Empty in this order). Returns seconds; *check
 * gets the sum of dequeued values (keeps the work observable). */
double cpu_ring_mixed(int64_t cap, int64_t n_ops, int64_t *check)
{
    int32_t *ring = malloc(sizeof(int32_t) * (size_t)cap);
    int64_t head = 0, tail = 0, sum = 0;
    double t0 = now_s();
    for (int64_t i = 0; i < n_ops; i++) {
        if ((i & 1) == 0) {
            if (tail - head < cap) {
                ring[tail % cap] = (int32_t)(i >> 1);
                tail++;
            }
        } else if (head < tail) {
            sum += ring[head % cap];
            head++;
        }
    }
    double t = now_s() - t0;
    free(ring);
    *check = sum;
    return t;
}

typedef struct {
    _Atomic int64_t count;
    char pad0[56];
    _Atomic uint64_t head;
    char pad1[56];
    _Atomic uint64_t tail;
    char pad2[56];
    _Atomic uint32_t *tickets;
    int32_t *ring;
    uint64_t n;      /* capacity, power of two */
    uint32_t log_n;
} bq_model;

/* ENSURE_ENQUEUE: reserve one slot on the broker count while it shows room */
static int ensure_enqueue(bq_model *q)
{
    int64_t num = atomic_load_explicit(&q->count, memory_order_relaxed);
    while (num < (int64_t)q->n) {
        if (atomic_fetch_add_explicit(&q->count, 1, memory_order_relaxed) < (int64_t)q->n)
            return 1;
        num = atomic_fetch_sub_explicit(&q->count, 1, memory_order_relaxed) - 1;
    }
    return 0;
}

/* ENSURE_DEQUEUE: the mirror image (a decrement whose old value was > 0) */
static int ensure_dequeue(bq_model *q)
{
    int64_t num = atomic_load_explicit(&q->count, memory_order_relaxed);
    while (num > 0) {
        if (atomic_fetch_sub_explicit(&q->count, 1, memory_order_relaxed) > 0)
            return 1;
        num = atomic_fetch_add_explicit(&q->count, 1, memory_order_relaxed) + 1;
    }
    return 0;
}

static void wait_ticket(_Atomic uint32_t *t, uint32_t want)
{
    int spins = 0;
    while (atomic_load_explicit(t, memory_order_acquire) != want)
        if (++spins > 64) {
            sched_yield();
            spins = 0;
        }
}

static int bq_enqueue(bq_model *q, int32_t v, int32_t *log)
{
    if (!ensure_enqueue(q))
        return 0;
    uint64_t pos = atomic_fetch_add_explicit(&q->tail, 1, memory_order_relaxed);
    uint64_t slot = pos & (q->n - 1);
    uint32_t r = (uint32_t)(pos >> q->log_n);
    wait_ticket(&q->tickets[slot], 2u * r);
    q->ring[slot] = v;
    atomic_store_explicit(&q->tickets[slot], 2u * r + 1u, memory_order_release);
    if (log)
        log[pos] = v;
    return 1;
}

static int bq_dequeue(bq_model *q, int32_t *out, int32_t *log)
{
    if (!ensure_dequeue(q))
        return 0;
    uint64_t pos = atomic_fetch_add_explicit(&q->head, 1, memory_order_relaxed);
    uint64_t slot = pos & (q->n - 1);
    uint32_t r = (uint32_t)(pos >> q->log_n);
    wait_ticket(&q->tickets[slot], 2u * r + 1u);
    int32_t v = q->ring[slot];
    atomic_store_explicit(&q->tickets[slot], 2u * (r + 1u), memory_order_release);
    if (log)
        log[pos] = v;
    *out = v;
    return 1;
}

typedef struct {
    bq_model *q;
    int64_t first, cnt; /* this thread's operations */
    int enq;
    int32_t *log;
    int64_t fails;
} worker;

static void *run_worker(void *arg)
{
    worker *w = arg;
    for (int64_t i = 0; i < w->cnt; i++) {
        int32_t v = (int32_t)(w->first + i), out;
        for (;;) {
            int ok = w->enq ? bq_enqueue(w->q, v, w->log) : bq_dequeue(w->q, &out, w->log);
            if (ok)
                break;
            w->fails++;
            sched_yield();
        }
    }
    return NULL;
}

/* Global Mixed on the host: `threads` threads (even: enqueuers, odd:
 * dequeuers), n_ops / 2 operations of each kind, value i for enqueue
 * operation i, each enqueuer thread taking a contiguous block of values.
 * enq_log / deq_log (NULL or int32[n_ops/2]) get the value at each position.
 * Returns seconds; *fails = Full / Empty attempts retried. */
double cpu_bq_mixed(int64_t cap, int64_t n_ops, int32_t threads, int32_t *enq_log,
                    int32_t *deq_log, int64_t *fails)
{
    bq_model q;
    memset(&q, 0, sizeof q);
    q.n = (uint64_t)cap;
    while ((1ull << q.log_n) < q.n)
        q.log_n++;
    q.tickets = calloc((size_t)cap, sizeof(_Atomic uint32_t));
    q.ring = calloc((size_t)cap, sizeof(int32_t));
    if (threads < 2)
        threads = 2;
    threads &= ~1;
    const int64_t half = n_ops / 2, per_role = threads / 2;
    worker *w = calloc((size_t)threads, sizeof(worker));
    pthread_t *tid = calloc((size_t)threads, sizeof(pthread_t));
    for (int32_t t = 0; t < threads; t++) {
        const int64_t k = t / 2;
        const int64_t lo = half * k / per_role, hi = half * (k + 1) / per_role;
        w[t].q = &q;
        w[t].first = lo;
        w[t].cnt = hi - lo;
        w[t].enq = (t & 1) == 0;
        w[t].log = w[t].enq ? enq_log : deq_log;
    }
    double t0 = now_s();
    for (int32_t t = 0; t < threads; t++)
        pthread_create(&tid[t], NULL, run_worker, &w[t]);
    for (int32_t t = 0; t < threads; t++)
        pthread_join(tid[t], NULL);
    double t = now_s() - t0;
    int64_t f = 0;
    for (int32_t i = 0; i < threads; i++)
        f += w[i].fails;
    *fails = f;
    free(w);
    free(tid);
    free(q.tickets);
    free(q.ring);
    return t;
}
