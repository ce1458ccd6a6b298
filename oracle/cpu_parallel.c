/*
 * Multi-core CPU baseline for the benchmark (test and measurement
 * infrastructure only, like the rest of this directory; not the parity
 * authority, which is the single-thread round form in oracle.c).
 *
 * The same rounds as Alg. 3 (relax every edge, count the changes, stop when
 * a round changes nothing, a change in round n-1 proves a negative cycle),
 * run as Jacobi rounds pulled over the transposed graph: in round i every
 * vertex v takes min(d[v], min over in-edges (u,v,w) of d[u] + w) from the
 * previous round's labels, one thread per block of vertices (OpenMP). After
 * round i the labels are the best walks of at most i+1 edges, so the result
 * and the negative-cycle decision equal the single-thread round form's.
 */
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define CPU_INF INT64_MAX

/* Transpose CSR (off, col, w) into CSC (toff[n+1], tsrc[m], tw[m]). */
void cpu_transpose(int32_t n, const int64_t *off, const int32_t *col, const int32_t *w,
                   int64_t *toff, int32_t *tsrc, int32_t *tw)
{
    int64_t m = off[n];
    memset(toff, 0, sizeof(int64_t) * ((size_t)n + 1));
    for (int64_t e = 0; e < m; e++)
        toff[col[e] + 1]++;
    for (int32_t v = 0; v < n; v++)
        toff[v + 1] += toff[v];
    int64_t *fill = malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    memcpy(fill, toff, sizeof(int64_t) * (size_t)n);
    for (int32_t u = 0; u < n; u++)
        for (int64_t e = off[u]; e < off[u + 1]; e++) {
            int64_t p = fill[col[e]]++;
            tsrc[p] = u;
            tw[p] = w[e];
        }
    free(fill);
}

/* Jacobi rounds over the transposed graph with all OpenMP threads.
 * Returns the rounds run; *neg as in oracle_bf_rounds; *threads = threads used. */
int64_t cpu_bf_jacobi(int32_t n, const int64_t *toff, const int32_t *tsrc, const int32_t *tw,
                      int32_t src, int64_t *d, int32_t *neg, int32_t *threads)
{
    int64_t *nd = malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    for (int32_t v = 0; v < n; v++)
        d[v] = CPU_INF;
    d[src] = 0;
    *neg = 0;
    *threads = omp_get_max_threads();
    int64_t rounds = 0;
    for (int64_t i = 0; i < n; i++) {
        int64_t changes = 0;
        rounds++;
#pragma omp parallel for schedule(dynamic, 4096) reduction(+ : changes)
        for (int32_t v = 0; v < n; v++) {
            int64_t best = d[v];
            for (int64_t e = toff[v]; e < toff[v + 1]; e++) {
                int64_t du = d[tsrc[e]];
                if (du != CPU_INF && du + (int64_t)tw[e] < best)
                    best = du + (int64_t)tw[e];
            }
            nd[v] = best;
            changes += best < d[v];
        }
        int64_t *t = d;
        memcpy(t, nd, sizeof(int64_t) * (size_t)n);
        if (changes == 0)
            break;
        if (i == (int64_t)n - 1)
            *neg = 1;
    }
    free(nd);
    return rounds;
}
