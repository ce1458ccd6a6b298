/* The host model of the Broker Queue (oracle/queue_cpu.c) under
 * ThreadSanitizer, built on its own by tests/test_sanitizers.py: Global
 * Mixed runs on several threads and capacities, each followed by the
 * position rule (the value read at position P is the value written at P)
 * and conservation (every value 0 .. n_ops/2 - 1 dequeued exactly once).
 * Exit status 0 when every check holds; ThreadSanitizer reports data races
 * on its own and exits non-zero. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

double cpu_bq_mixed(int64_t cap, int64_t n_ops, int32_t threads, int32_t *enq_log,
                    int32_t *deq_log, int64_t *fails);

static int check(int64_t cap, int64_t n_ops, int32_t threads)
{
    const int64_t half = n_ops / 2;
    int32_t *el = malloc(sizeof(int32_t) * (size_t)half);
    int32_t *dl = malloc(sizeof(int32_t) * (size_t)half);
    char *seen = calloc((size_t)half, 1);
    int64_t fails = 0;
    for (int64_t i = 0; i < half; i++)
        el[i] = dl[i] = -1;
    cpu_bq_mixed(cap, n_ops, threads, el, dl, &fails);
    int bad = 0;
    for (int64_t p = 0; p < half && !bad; p++) {
        if (el[p] != dl[p]) {
            fprintf(stderr, "cap %lld: position %lld enqueued %d dequeued %d\n", (long long)cap,
                    (long long)p, el[p], dl[p]);
            bad = 1;
        } else if (dl[p] < 0 || dl[p] >= half || seen[dl[p]]++) {
            fprintf(stderr, "cap %lld: value %d lost or repeated\n", (long long)cap, dl[p]);
            bad = 1;
        }
    }
    free(el);
    free(dl);
    free(seen);
    return bad;
}

int main(void)
{
    const int64_t caps[] = {1, 2, 64, 4096};
    const int32_t threads[] = {2, 4, 8};
    for (unsigned i = 0; i < sizeof caps / sizeof caps[0]; i++)
        for (unsigned j = 0; j < sizeof threads / sizeof threads[0]; j++)
            if (check(caps[i], 1 << 13, threads[j]))
                return 1;
    printf("queue model ok\n");
    return 0;
}
