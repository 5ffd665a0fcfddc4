/*
 * Brute-force enumerators used to pin the oracle.  TEST INFRASTRUCTURE ONLY.
 *
 * Nothing here propagates: constraints are only *checked* on (partial)
 * assignments, straight from their definitions.  This file shares no code
 * with propagate.c / search.c, so a mistake in a propagator cannot hide in
 * both.
 *
 *  - orc_brute_points: every integer point of the initial box that satisfies
 *    every linear row (sum a_t x_t <= c) and every reified item
 *    ((b >= 1) <=> (si <= sj and sj < si + d)).  Variables are assigned in
 *    index order; a partial assignment is abandoned only when a row cannot
 *    be satisfied whatever values the unassigned variables take in their
 *    boxes, so no solution is skipped.  Guarded commands are checked on
 *    complete points only, as the constraint they state: when every guard
 *    holds (y >= c, or y <= c), div * x >= k + sum a_t y_t for an lb tell,
 *    div * x <= k + sum a_t y_t for an ub tell.
 *  - orc_brute_rcpsp: the RCPSP of §2 stated on raw data (durations,
 *    precedences, demands, capacities), independent of the Boolean
 *    decomposition: s_i + d_i <= s_j for each precedence, and at every
 *    instant t the tasks running at t (s_i <= t < s_i + d_i) use at most c_k
 *    of each resource k.  The makespan is max_i (s_i + d_i).
 */
#include "oracle.h"

#include <limits.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

uint64_t orc_solution_hash(const int32_t *vals, int32_t n);

typedef struct {
    const orc_model *m;
    int32_t *x;                 /* current assignment                      */
    int32_t **rows_of;          /* rows containing each variable           */
    int32_t *nrows_of;
    int32_t **reif_of;          /* reified items whose largest var is v     */
    int32_t *nreif_of;
    int32_t *vals;
    int32_t *out;
    int64_t cap, count;
    uint64_t hash;
} bctx;

/* can row r still hold if variables >= k+1 take any value in their box? */
static int row_possible(const bctx *c, int32_t r, int32_t k)
{
    const orc_model *m = c->m;
    int64_t tot = 0;
    for (int32_t t = m->row_ptr[r]; t < m->row_ptr[r + 1]; ++t) {
        int32_t v = m->var[t];
        int64_t a = m->coef[t];
        if (v <= k) {
            tot += a * c->x[v];
        } else {
            int64_t lo = a * m->lb0[v], hi = a * m->ub0[v];
            tot += lo < hi ? lo : hi;
        }
    }
    return tot <= m->rhs[r];
}

static int reif_holds(const int32_t *x, const int32_t *it)
{
    int64_t b = x[it[0]], si = x[it[1]], sj = x[it[2]], d = it[3];
    int psi = (si <= sj) && (sj < si + d);
    return (b >= 1) == psi;
}

static int cmd_holds(const orc_model *m, const int32_t *x, int32_t q)
{
    for (int32_t g = m->cmd_gptr[q]; g < m->cmd_gptr[q + 1]; ++g) {
        const int32_t *gd = m->guard + 3 * (int64_t)g;
        const int holds = gd[1] == 0 ? x[gd[0]] >= gd[2] : x[gd[0]] <= gd[2];
        if (!holds)
            return 1;          /* a guard is false: the command states nothing */
    }
    const int32_t *cm = m->cmd + 4 * (int64_t)q;
    int64_t f = cm[2];
    for (int32_t t = m->cmd_tptr[q]; t < m->cmd_tptr[q + 1]; ++t)
        f += (int64_t)m->cterm[2 * (int64_t)t] * x[m->cterm[2 * (int64_t)t + 1]];
    const int64_t lhs = (int64_t)cm[3] * x[cm[0]];
    return cm[1] == 0 ? lhs >= f : lhs <= f;
}

static void brute_rec(bctx *c, int32_t k)
{
    const orc_model *m = c->m;
    if (k == m->nvars) {
        for (int32_t q = 0; q < m->ncmd; ++q)
            if (!cmd_holds(m, c->x, q))
                return;
        for (int32_t q = 0; q < m->ndec; ++q)
            c->vals[q] = c->x[m->dec[q]];
        if (c->out && c->count < c->cap)
            memcpy(c->out + c->count * (int64_t)m->ndec, c->vals,
                   sizeof(int32_t) * (size_t)m->ndec);
        c->hash += orc_solution_hash(c->vals, m->ndec);
        c->count += 1;
        return;
    }
    for (int64_t val = m->lb0[k]; val <= m->ub0[k]; ++val) {
        c->x[k] = (int32_t)val;
        int ok = 1;
        for (int32_t q = 0; q < c->nrows_of[k] && ok; ++q)
            ok = row_possible(c, c->rows_of[k][q], k);
        for (int32_t q = 0; q < c->nreif_of[k] && ok; ++q)
            ok = reif_holds(c->x, m->reif + 4 * (int64_t)c->reif_of[k][q]);
        if (ok)
            brute_rec(c, k + 1);
    }
}

int64_t orc_brute_points(const orc_model *m, int32_t *out, int64_t cap, uint64_t *hash)
{
    if (orc_validate(m) != 0)
        return -1;
    const int32_t V = m->nvars;
    bctx c;
    memset(&c, 0, sizeof(c));
    c.m = m;
    c.out = out;
    c.cap = out ? cap : 0;
    c.x = (int32_t *)calloc((size_t)(V + 1), sizeof(int32_t));
    c.vals = (int32_t *)calloc((size_t)(m->ndec + 1), sizeof(int32_t));
    c.rows_of = (int32_t **)calloc((size_t)(V + 1), sizeof(int32_t *));
    c.nrows_of = (int32_t *)calloc((size_t)(V + 1), sizeof(int32_t));
    c.reif_of = (int32_t **)calloc((size_t)(V + 1), sizeof(int32_t *));
    c.nreif_of = (int32_t *)calloc((size_t)(V + 1), sizeof(int32_t));
    for (int32_t v = 0; v < V; ++v) {
        c.rows_of[v] = (int32_t *)malloc(sizeof(int32_t) * (size_t)(m->nrows + 1));
        c.reif_of[v] = (int32_t *)malloc(sizeof(int32_t) * (size_t)(m->nreif + 1));
    }
    for (int32_t r = 0; r < m->nrows; ++r)
        for (int32_t t = m->row_ptr[r]; t < m->row_ptr[r + 1]; ++t) {
            int32_t v = m->var[t];
            c.rows_of[v][c.nrows_of[v]++] = r;
        }
    for (int32_t q = 0; q < m->nreif; ++q) {
        const int32_t *it = m->reif + 4 * (int64_t)q;
        int32_t mx = it[0];
        if (it[1] > mx) mx = it[1];
        if (it[2] > mx) mx = it[2];
        c.reif_of[mx][c.nreif_of[mx]++] = q;
    }
    int empty = 0;
    for (int32_t v = 0; v < V; ++v)
        if (m->lb0[v] > m->ub0[v])
            empty = 1;
    if (!empty)
        brute_rec(&c, 0);
    for (int32_t v = 0; v < V; ++v) {
        free(c.rows_of[v]);
        free(c.reif_of[v]);
    }
    free(c.rows_of);
    free(c.nrows_of);
    free(c.reif_of);
    free(c.nreif_of);
    free(c.x);
    free(c.vals);
    if (hash)
        *hash = c.hash;
    return c.count;
}

/* ---------------------------------------------------------------------- */
int32_t orc_check_schedule(int32_t n, const int32_t *dur, int32_t nedges,
                           const int32_t *edges, int32_t nres,
                           const int32_t *dem, const int32_t *cap,
                           const int32_t *s, int32_t *makespan)
{
    int64_t ms = 0;
    for (int32_t i = 0; i < n; ++i) {
        if (s[i] < 0)
            return 0;
        if ((int64_t)s[i] + dur[i] > ms)
            ms = (int64_t)s[i] + dur[i];
    }
    if (makespan)
        *makespan = (int32_t)ms;
    for (int32_t e = 0; e < nedges; ++e) {
        int32_t i = edges[2 * e], j = edges[2 * e + 1];
        if ((int64_t)s[i] + dur[i] > s[j])
            return 0;
    }
    for (int64_t t = 0; t < ms; ++t)
        for (int32_t k = 0; k < nres; ++k) {
            int64_t use = 0;
            for (int32_t i = 0; i < n; ++i)
                if (s[i] <= t && t < (int64_t)s[i] + dur[i])
                    use += dem[(int64_t)k * n + i];
            if (use > cap[k])
                return 0;
        }
    return 1;
}

typedef struct {
    int32_t n, nedges, nres, h;
    const int32_t *dur, *edges, *dem, *cap;
    int32_t *s, *best_s;
    int32_t best;
} rctx;

static void rcpsp_rec(rctx *c, int32_t j)
{
    if (j == c->n) {
        int32_t ms;
        if (orc_check_schedule(c->n, c->dur, c->nedges, c->edges, c->nres, c->dem,
                               c->cap, c->s, &ms) && ms < c->best) {
            c->best = ms;
            if (c->best_s)
                memcpy(c->best_s, c->s, sizeof(int32_t) * (size_t)c->n);
        }
        return;
    }
    /* partial check: every precedence into j from an already placed task */
    int64_t est = 0;
    for (int32_t e = 0; e < c->nedges; ++e) {
        int32_t i = c->edges[2 * e], jj = c->edges[2 * e + 1];
        if (jj == j && i < j && (int64_t)c->s[i] + c->dur[i] > est)
            est = (int64_t)c->s[i] + c->dur[i];
    }
    for (int64_t v = est; v + c->dur[j] <= c->h; ++v) {
        c->s[j] = (int32_t)v;
        rcpsp_rec(c, j + 1);
    }
}

int32_t orc_brute_rcpsp(int32_t n, const int32_t *dur, int32_t nedges,
                        const int32_t *edges, int32_t nres, const int32_t *dem,
                        const int32_t *cap, int32_t h, int32_t *best_s)
{
    /* the partial check needs every edge to go from a lower to a higher
     * task index (the generator's edges do) */
    for (int32_t e = 0; e < nedges; ++e)
        if (edges[2 * e] >= edges[2 * e + 1])
            return -2;
    rctx c = {n, nedges, nres, h, dur, edges, dem, cap, NULL, best_s, INT32_MAX};
    c.s = (int32_t *)calloc((size_t)(n + 1), sizeof(int32_t));
    rcpsp_rec(&c, 0);
    free(c.s);
    return c.best == INT32_MAX ? -1 : c.best;
}
