/*
 * CPU oracle for the queue-driven Bellman-Ford path.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing on the product path may call, link or
 * load this file: only the tests, the smoke check and the benchmark's CPU
 * baseline leg do. It shares no code, header, table or helper with the HIP
 * library; both sides get their inputs from the seeded generators alone.
 *
 * Plain, slow, single-threaded C over int64 distances. Each function says
 * which part of the paper it follows.
 *
 * Graph format: CSR, off[n+1] (int64), col[m] (int32), w[m] (int32);
 * distances int64 with INF = INT64_MAX for "not reached" (the paper's
 * infinity in Alg. 3's INITIALIZE_DISTRIBUTED_DISTANCES).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_INF INT64_MAX

/* Alg. 3, INITIALIZE_DISTRIBUTED_DISTANCES: source 0, every other vertex
 * infinity. */
static void init_distances(int32_t n, int32_t src, int64_t *d)
{
    for (int32_t v = 0; v < n; v++)
        d[v] = ORACLE_INF;
    d[src] = 0;
}

/*
 * Round-based Bellman-Ford on one processing element: Alg. 3's
 * MULTI_GPU_BELLMANFORD with a single GPU, i.e. repeated passes of
 * PARALLEL_RELAX_EDGES over every edge, with its relax rule (skip a source at
 * infinity; lower the target when source + weight is smaller; count the
 * change), the change counter's early exit (Section III.C) and the
 * negative-cycle rule (changes in the round indexed n-1).
 *
 * Readings where the text is loose: the rounds are indexed 0..n-1 and the
 * counter is reset at the start of each round; updates are in place, so a
 * later edge of the same round sees an earlier edge's update (the single-PE
 * case of the put in PARALLEL_RELAX_EDGES); edges are visited in CSR order.
 *
 * Returns the number of rounds run. *neg = 1 when a negative cycle is
 * reachable from src; d is then not meaningful.
 */
int64_t oracle_bf_rounds(int32_t n, const int64_t *off, const int32_t *col,
                         const int32_t *w, int32_t src, int64_t *d,
                         int32_t *neg)
{
    init_distances(n, src, d);
    *neg = 0;
    int64_t rounds = 0;
    for (int64_t i = 0; i < n; i++) {
        int64_t changes = 0;
        rounds++;
        for (int32_t u = 0; u < n; u++) {
            for (int64_t e = off[u]; e < off[u + 1]; e++) {
                int64_t dist1 = d[u];
                int32_t v = col[e];
                if (dist1 != ORACLE_INF) {
                    int64_t nd = dist1 + (int64_t)w[e];
                    if (nd < d[v]) {
                        d[v] = nd;
                        changes++;
                    }
                }
            }
        }
        if (changes == 0)
            break;
        if (i == (int64_t)n - 1 && changes > 0)
            *neg = 1;
    }
    return rounds;
}

/*
 * Sequential FIFO Bellman-Ford (the single-thread form of the queue-based
 * method of Section III.C): a FIFO seeded with src; pop u; relax each
 * out-edge of u with d[u] read when u is popped; push every target whose
 * distance dropped and that is not already in the queue.
 *
 * Negative cycles: a label that needed n or more edges can only come from a
 * walk that repeats a vertex, and with no negative cycle such a walk never
 * strictly lowers a label, so hops >= n proves a negative cycle (textbook
 * argument, sound and complete). As a faster trigger the parent graph (each
 * vertex points at the edge that set its label) is searched for a cycle
 * after every n pops; a cycle found there is accepted only if the weights of
 * its edges sum to a negative number, which is a certificate on its own.
 *
 * The queue is a ring of capacity n: a vertex is in it at most once.
 * Returns the number of pops. *relax counts edge relaxations (edges scanned).
 */
static int parent_cycle_negative(int32_t n, const int32_t *col,
                                 const int32_t *w, const int64_t *pedge,
                                 const int32_t *psrc, uint8_t *mark);

int64_t oracle_bf_fifo(int32_t n, const int64_t *off, const int32_t *col,
                       const int32_t *w, int32_t src, int64_t *d,
                       int32_t *neg, int64_t *relax)
{
    int32_t *ring = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    uint8_t *inq = (uint8_t *)calloc((size_t)n, 1);
    int32_t *hops = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int64_t *pedge = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    int32_t *psrc = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    uint8_t *mark = (uint8_t *)malloc((size_t)n);
    init_distances(n, src, d);
    for (int32_t v = 0; v < n; v++) {
        pedge[v] = -1;
        psrc[v] = -1;
    }
    hops[src] = 0;
    *neg = 0;
    *relax = 0;
    int64_t head = 0, size = 0, pops = 0;
    ring[0] = src;
    inq[src] = 1;
    size = 1;
    while (size > 0) {
        int32_t u = ring[head];
        head = (head + 1 == n) ? 0 : head + 1;
        size--;
        inq[u] = 0;
        pops++;
        int64_t du = d[u];
        int32_t hu = hops[u];
        for (int64_t e = off[u]; e < off[u + 1]; e++) {
            int32_t v = col[e];
            int64_t nd = du + (int64_t)w[e];
            (*relax)++;
            if (nd < d[v]) {
                d[v] = nd;
                hops[v] = hu + 1;
                pedge[v] = e;
                psrc[v] = u;
                if (hops[v] >= n) {
                    *neg = 1;
                    goto done;
                }
                if (!inq[v]) {
                    int64_t tail = head + size;
                    if (tail >= n)
                        tail -= n;
                    ring[tail] = v;
                    size++;
                    inq[v] = 1;
                }
            }
        }
        if (pops % n == 0 && parent_cycle_negative(n, col, w, pedge, psrc, mark)) {
            *neg = 1;
            goto done;
        }
    }
done:
    free(ring);
    free(inq);
    free(hops);
    free(pedge);
    free(psrc);
    free(mark);
    return pops;
}

/* Walk the parent graph (v -> psrc[v]) from every unvisited vertex; mark 1 =
 * on the current walk, 2 = finished. A walk that meets its own mark closes a
 * cycle; sum the weights of the parent edges around it. */
static int parent_cycle_negative(int32_t n, const int32_t *col,
                                 const int32_t *w, const int64_t *pedge,
                                 const int32_t *psrc, uint8_t *mark)
{
    (void)col;
    memset(mark, 0, (size_t)n);
    for (int32_t s = 0; s < n; s++) {
        if (mark[s])
            continue;
        int32_t x = s;
        while (x >= 0 && mark[x] == 0) {
            mark[x] = 1;
            x = psrc[x];
        }
        if (x >= 0 && mark[x] == 1) {
            int64_t sum = 0;
            int32_t y = x;
            do {
                sum += w[pedge[y]];
                y = psrc[y];
            } while (y != x);
            if (sum < 0)
                return 1;
        }
        x = s;
        while (x >= 0 && mark[x] == 1) {
            mark[x] = 2;
            x = psrc[x];
        }
    }
    return 0;
}

/*
 * Predecessors: for every reached v other than src, the smallest vertex id u
 * among v's in-neighbours with d[u] finite and d[u] + w(u,v) == d[v]; -1 for
 * src and for unreached vertices. The paper returns only distances (Alg. 3's
 * output); this fixes one of the equally valid shortest-path trees so that
 * predecessors can be compared exactly.
 */
void oracle_pred(int32_t n, const int64_t *off, const int32_t *col,
                 const int32_t *w, int32_t src, const int64_t *d,
                 int32_t *pred)
{
    for (int32_t v = 0; v < n; v++)
        pred[v] = -1;
    for (int32_t u = 0; u < n; u++) {
        if (d[u] == ORACLE_INF)
            continue;
        for (int64_t e = off[u]; e < off[u + 1]; e++) {
            int32_t v = col[e];
            if (v == src)
                continue;
            if (d[u] + (int64_t)w[e] == d[v] && (pred[v] < 0 || u < pred[v]))
                pred[v] = u;
        }
    }
}

/*
 * Minus-infinity marking (beyond the paper, which only detects): the
 * distance of v is minus infinity exactly when v is reachable from a negative
 * cycle that src reaches, because a walk to v can then go round the cycle
 * as often as wanted. The textbook way to find these vertices with rounds:
 *  1. n-1 rounds of the round form (oracle_bf_rounds' relax rule, stopping
 *     early when a round changes nothing). Afterwards every vertex that no
 *     negative cycle reaches holds its exact distance (a shortest simple
 *     path has at most n-1 edges) and no label is below the true distance.
 *  2. Mark v when some edge u->v with d[u] finite still lowers d[v]: then
 *     d[v] is not exact, so a negative cycle reaches v. Every reachable
 *     negative cycle has such an edge, since the slacks d[u] + w - d[v]
 *     round the cycle sum to its (negative) weight.
 *  3. Spread the marks along edges, round by round, until nothing changes.
 * Output: mark[v] = 1 for the minus-infinity vertices; d holds the labels
 * of step 1 (exact for unmarked vertices, INF for unreached ones).
 * Returns the number of marked vertices.
 */
int64_t oracle_neg_inf(int32_t n, const int64_t *off, const int32_t *col,
                       const int32_t *w, int32_t src, int64_t *d,
                       int8_t *mark)
{
    init_distances(n, src, d);
    for (int64_t i = 0; i + 1 < n; i++) {
        int64_t changes = 0;
        for (int32_t u = 0; u < n; u++) {
            if (d[u] == ORACLE_INF)
                continue;
            for (int64_t e = off[u]; e < off[u + 1]; e++) {
                int64_t nd = d[u] + (int64_t)w[e];
                if (nd < d[col[e]]) {
                    d[col[e]] = nd;
                    changes++;
                }
            }
        }
        if (changes == 0)
            break;
    }
    for (int32_t v = 0; v < n; v++)
        mark[v] = 0;
    for (int32_t u = 0; u < n; u++) {
        if (d[u] == ORACLE_INF)
            continue;
        for (int64_t e = off[u]; e < off[u + 1]; e++)
            if (d[u] + (int64_t)w[e] < d[col[e]])
                mark[col[e]] = 1;
    }
    int64_t grew = 1;
    while (grew) {
        grew = 0;
        for (int32_t u = 0; u < n; u++) {
            if (!mark[u])
                continue;
            for (int64_t e = off[u]; e < off[u + 1]; e++)
                if (!mark[col[e]]) {
                    mark[col[e]] = 1;
                    grew = 1;
                }
        }
    }
    int64_t total = 0;
    for (int32_t v = 0; v < n; v++)
        total += mark[v];
    return total;
}

/*
 * Sequential bounded FIFO of capacity cap (the sequential specification the
 * concurrent queue must be linearizable to; Section II.B and the queue of
 * Section III.A): enqueue fails (Full) iff it holds cap items, dequeue fails
 * (Empty) iff it holds none, otherwise the oldest item leaves first.
 *
 * ops[i] >= 0 enqueues that value; ops[i] < 0 requests one dequeue.
 * res[i] = 1 / 0 for enqueue success / Full; for dequeue, out[i] gets the
 * value and res[i] = 1, or res[i] = 0 on Empty. Returns the final size.
 */
int64_t oracle_fifo_run(int64_t cap, int64_t nops, const int64_t *ops,
                        int8_t *res, int64_t *out)
{
    int64_t *ring = (int64_t *)malloc(sizeof(int64_t) * (size_t)(cap > 0 ? cap : 1));
    int64_t head = 0, size = 0;
    for (int64_t i = 0; i < nops; i++) {
        out[i] = -1;
        if (ops[i] >= 0) {
            if (size == cap) {
                res[i] = 0;
            } else {
                ring[(head + size) % cap] = ops[i];
                size++;
                res[i] = 1;
            }
        } else {
            if (size == 0) {
                res[i] = 0;
            } else {
                out[i] = ring[head];
                head = (head + 1) % cap;
                size--;
                res[i] = 1;
            }
        }
    }
    free(ring);
    return size;
}
