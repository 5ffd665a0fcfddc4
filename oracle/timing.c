/*
 * CPU oracle: timing harness for the CPU baseline.  TEST INFRASTRUCTURE
 * ONLY (see oracle.h); never linked into the product.
 *
 * Runs the sequential search of search.c (orc_solve, unchanged) on
 * independent instances, one POSIX thread per host core, each thread taking
 * the next unsolved instance from a shared counter.  Times are taken in C
 * with CLOCK_MONOTONIC (the C counterpart of a steady clock), around each
 * instance and around the whole set, so that no interpreter time is counted.
 */
#define _POSIX_C_SOURCE 200809L
#include "oracle.h"

#include <pthread.h>
#include <stdatomic.h>
#include <stdlib.h>
#include <time.h>

static double now_s(void)
{
    struct timespec t;
    clock_gettime(CLOCK_MONOTONIC, &t);
    return (double)t.tv_sec + 1e-9 * (double)t.tv_nsec;
}

typedef struct {
    const orc_model *const *models;
    int32_t n, mode, branching;
    int64_t node_limit;
    int64_t *nodes;
    double *secs;
    int32_t *outcome, *best;
    atomic_int next;
    atomic_int err;
} timed_job;

static void *worker(void *arg)
{
    timed_job *j = (timed_job *)arg;
    for (;;) {
        const int i = atomic_fetch_add(&j->next, 1);
        if (i >= j->n) break;
        orc_stats st;
        const double t0 = now_s();
        const int32_t rc = orc_solve(j->models[i], j->mode, j->branching, j->node_limit,
                                     NULL, 0, NULL, &st);
        j->secs[i] = now_s() - t0;
        if (rc < 0) {
            atomic_store(&j->err, rc);
            continue;
        }
        j->nodes[i] = st.nodes;
        j->outcome[i] = st.outcome;
        j->best[i] = st.best;
    }
    return NULL;
}

int32_t orc_solve_timed(const orc_model *const *models, int32_t n, int32_t mode,
                        int32_t branching, int64_t node_limit, int32_t threads,
                        int64_t *nodes, double *secs, int32_t *outcome, int32_t *best,
                        double *wall_s)
{
    if (!models || n < 0 || threads < 1 || !nodes || !secs || !outcome || !best || !wall_s)
        return -1;
    timed_job j;
    j.models = models;
    j.n = n;
    j.mode = mode;
    j.branching = branching;
    j.node_limit = node_limit;
    j.nodes = nodes;
    j.secs = secs;
    j.outcome = outcome;
    j.best = best;
    atomic_init(&j.next, 0);
    atomic_init(&j.err, 0);
    if (threads > n) threads = n > 0 ? n : 1;
    pthread_t *th = (pthread_t *)calloc((size_t)threads, sizeof(pthread_t));
    if (!th) return -1;
    const double t0 = now_s();
    int started = 0;
    for (; started < threads; ++started)
        if (pthread_create(&th[started], NULL, worker, &j) != 0) break;
    if (started == 0) worker(&j);
    for (int k = 0; k < started; ++k) pthread_join(th[k], NULL);
    *wall_s = now_s() - t0;
    free(th);
    return atomic_load(&j.err);
}
