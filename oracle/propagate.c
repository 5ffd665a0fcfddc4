/*
 * CPU oracle: propagators and the propagation loop.  TEST INFRASTRUCTURE
 * ONLY (see oracle.h); never linked into the product.
 *
 * Every guarded command of the model is one of:
 *   - a term of a linear row  sum_t a_t x_t <= c  (the tell on x_t),
 *   - one of the ten tells of a reified overlap item, or
 *   - a general guarded command of the model (its own propagator).
 * A propagator is one row or one reified item (§2, the function [[.]] maps a
 * constraint to a process).  The guarded normal form of §3 (gnf) flattens a
 * propagator into its commands; the commands are listed below in the order
 * the sequential schedule executes them.
 */
#include "oracle.h"

#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------------- */
/* integer division rounding toward -infinity / +infinity (b != 0).  C's '/'
 * truncates toward zero, which is wrong for negative quotients.            */
static int64_t floor_div(int64_t a, int64_t b)
{
    int64_t q = a / b, r = a % b;
    if (r != 0 && ((r < 0) != (b < 0)))
        q -= 1;
    return q;
}

static int64_t ceil_div(int64_t a, int64_t b)
{
    return -floor_div(-a, b);
}

/* exported for the unit tests of the rounding helpers */
int64_t orc_floor_div(int64_t a, int64_t b) { return floor_div(a, b); }
int64_t orc_ceil_div(int64_t a, int64_t b) { return ceil_div(a, b); }

/* ---------------------------------------------------------------------- */
/* Tell = join of one bound into the store (§2, embed of a tell).  Returns
 * 1 if the store became strictly greater, 0 if unchanged; sets *failed when
 * the interval becomes empty (lb > ub): the store is then top.             */
typedef struct {
    int32_t *lb, *ub;
    int failed;
    int changed;
} store_t;

static void tell_lb(store_t *s, int32_t x, int64_t v)
{
    if (v > s->lb[x]) {
        s->lb[x] = (int32_t)v;
        s->changed = 1;
        if (s->lb[x] > s->ub[x])
            s->failed = 1;
    }
}

static void tell_ub(store_t *s, int32_t x, int64_t v)
{
    if (v < s->ub[x]) {
        s->ub[x] = (int32_t)v;
        s->changed = 1;
        if (s->lb[x] > s->ub[x])
            s->failed = 1;
    }
}

/* ---------------------------------------------------------------------- */
/* Linear row  sum_t a_t * x_t <= c  (§2: [[x + y <= c]] tells x the bound
 * c - lb(y); the resource sum tells b the bound given by the other terms).
 * The smallest value of term t over the box is m_t = a_t*lb(x_t) for
 * a_t > 0 and a_t*ub(x_t) for a_t < 0; with S = sum_t m_t the tell on x_t
 * is  a_t * x_t <= c - (S - m_t).                                          */
static int64_t term_min(const store_t *s, int32_t a, int32_t x)
{
    return a > 0 ? (int64_t)a * s->lb[x] : (int64_t)a * s->ub[x];
}

static void tell_term(store_t *s, int32_t a, int32_t x, int64_t rest_min, int64_t c)
{
    int64_t r = c - rest_min;             /* a * x <= r */
    if (a > 0)
        tell_ub(s, x, floor_div(r, a));
    else
        tell_lb(s, x, ceil_div(-r, -(int64_t)a));
}

/* all tells of one row; S is the same for every term because a row's tells
 * only move ub of positive-coefficient terms and lb of negative ones, which
 * are not the bounds S reads (variables are distinct within a row). */
static void run_row(const orc_model *m, store_t *s, int32_t r)
{
    int32_t a0 = m->row_ptr[r], a1 = m->row_ptr[r + 1];
    int64_t S = 0;
    for (int32_t t = a0; t < a1; ++t)
        S += term_min(s, m->coef[t], m->var[t]);
    for (int32_t t = a0; t < a1 && !s->failed; ++t) {
        int64_t mt = term_min(s, m->coef[t], m->var[t]);
        tell_term(s, m->coef[t], m->var[t], S - mt, m->rhs[r]);
    }
}

/* one term's tell on its own (used by the random single-command schedule) */
static void run_row_term(const orc_model *m, store_t *s, int32_t r, int32_t t)
{
    int32_t a0 = m->row_ptr[r], a1 = m->row_ptr[r + 1];
    int64_t rest = 0;
    for (int32_t u = a0; u < a1; ++u)
        if (u != t)
            rest += term_min(s, m->coef[u], m->var[u]);
    tell_term(s, m->coef[t], m->var[t], rest, m->rhs[r]);
}

/* ---------------------------------------------------------------------- */
/* Reified overlap  b <=> psi,  psi = (si <= sj) and (sj < si + d).
 * §2 compiles phi <=> psi into four guarded processes:
 *   if entailed(b)      then [[psi]]     if entailed(psi)  then [[b]]
 *   if entailed(not b)  then [[not psi]] if entailed(not psi) then [[not b]]
 * Entailment over intervals (§2 gives entailed(x + y <= c) = ub(x)+ub(y) <= c):
 *   E1 = entailed(si <= sj)       : ub(si) <= lb(sj)
 *   E2 = entailed(sj < si + d)    : ub(sj) <= lb(si) + d - 1
 *   N1 = entailed(not si <= sj)   : lb(si) >  ub(sj)
 *   N2 = entailed(not sj < si + d): lb(sj) >= ub(si) + d
 *   entailed(psi) = E1 and E2;  entailed(not psi) = N1 or N2
 *   entailed(b) = lb(b) >= 1;   entailed(not b) = ub(b) <= 0
 * [[psi]] = [[si - sj <= 0]] || [[sj - si <= d - 1]]  (§2, [[phi and psi]]).
 * not psi = (sj - si <= -1) or (si - sj <= -d): when one disjunct is
 * entailed false, the other is told.  The ten commands, in schedule order:
 *   0  E1 & E2          => lb(b)  >= 1
 *   1  N1 | N2          => ub(b)  <= 0
 *   2  lb(b) >= 1       => ub(si) <= ub(sj)
 *   3  lb(b) >= 1       => lb(sj) >= lb(si)
 *   4  lb(b) >= 1       => ub(sj) <= ub(si) + d - 1
 *   5  lb(b) >= 1       => lb(si) >= lb(sj) - d + 1
 *   6  ub(b) <= 0 & E1  => lb(sj) >= lb(si) + d
 *   7  ub(b) <= 0 & E1  => ub(si) <= ub(sj) - d
 *   8  ub(b) <= 0 & E2  => ub(sj) <= ub(si) - 1
 *   9  ub(b) <= 0 & E2  => lb(si) >= lb(sj) + 1                           */
#define REIF_NCMD 10

static void run_reif_cmd(store_t *s, const int32_t *it, int k)
{
    const int32_t b = it[0], i = it[1], j = it[2];
    const int64_t d = it[3];
    const int32_t *lb = s->lb, *ub = s->ub;
    const int E1 = (int64_t)ub[i] <= (int64_t)lb[j];
    const int E2 = (int64_t)ub[j] <= (int64_t)lb[i] + d - 1;
    switch (k) {
    case 0:
        if (E1 && E2) tell_lb(s, b, 1);
        break;
    case 1: {
        const int N1 = (int64_t)lb[i] > (int64_t)ub[j];
        const int N2 = (int64_t)lb[j] >= (int64_t)ub[i] + d;
        if (N1 || N2) tell_ub(s, b, 0);
        break;
    }
    case 2: if (lb[b] >= 1) tell_ub(s, i, ub[j]); break;
    case 3: if (lb[b] >= 1) tell_lb(s, j, lb[i]); break;
    case 4: if (lb[b] >= 1) tell_ub(s, j, (int64_t)ub[i] + d - 1); break;
    case 5: if (lb[b] >= 1) tell_lb(s, i, (int64_t)lb[j] - d + 1); break;
    case 6: if (ub[b] <= 0 && E1) tell_lb(s, j, (int64_t)lb[i] + d); break;
    case 7: if (ub[b] <= 0 && E1) tell_ub(s, i, (int64_t)ub[j] - d); break;
    case 8: if (ub[b] <= 0 && E2) tell_ub(s, j, (int64_t)ub[i] - 1); break;
    case 9: if (ub[b] <= 0 && E2) tell_lb(s, i, (int64_t)lb[j] + 1); break;
    }
}

static void run_reif(const orc_model *m, store_t *s, int32_t q)
{
    const int32_t *it = m->reif + 4 * (int64_t)q;
    for (int k = 0; k < REIF_NCMD && !s->failed; ++k)
        run_reif_cmd(s, it, k);
}

/* ---------------------------------------------------------------------- */
/* General guarded command  {g_1, ..., g_n} => x <- f  (§3: a command of the
 * guarded normal form; §2: "if b then P" runs P once b is true, and the
 * sugar "if e then P" first tells b <- e).  A guard is the entailment of a
 * bound constraint: entailed(y >= c) = lb(y) >= c, entailed(y <= c) =
 * ub(y) <= c (monotone by the lemma of §2 on partial orders as functions).
 * The tell is the join of f = k + sum_t a_t * y_t into one bound of x, where
 * every y_t is read through the bound that makes f move in the direction of
 * the join as the store grows (§2: tells must be monotone):
 *   lb tell: a_t > 0 reads lb(y_t), a_t < 0 reads ub(y_t); value ceil(f/div)
 *   ub tell: a_t > 0 reads ub(y_t), a_t < 0 reads lb(y_t); value floor(f/div)
 * Read as a constraint on points, the command says "if every guard holds,
 * div * x >= k + sum a_t y_t" (lb tell) or "<=" (ub tell); the bound read
 * through is the least (resp. greatest) value of the sum over the box, so
 * the tell removes no point that satisfies it.                             */
static int cmd_guards_hold(const orc_model *m, const store_t *s, int32_t q)
{
    for (int32_t g = m->cmd_gptr[q]; g < m->cmd_gptr[q + 1]; ++g) {
        const int32_t *gd = m->guard + 3 * (int64_t)g;
        if (gd[1] == 0 ? !(s->lb[gd[0]] >= gd[2]) : !(s->ub[gd[0]] <= gd[2]))
            return 0;
    }
    return 1;
}

static void run_cmd(const orc_model *m, store_t *s, int32_t q)
{
    if (!cmd_guards_hold(m, s, q))
        return;
    const int32_t *c = m->cmd + 4 * (int64_t)q;
    const int32_t x = c[0], side = c[1];
    int64_t f = c[2];
    for (int32_t t = m->cmd_tptr[q]; t < m->cmd_tptr[q + 1]; ++t) {
        const int64_t a = m->cterm[2 * (int64_t)t];
        const int32_t y = m->cterm[2 * (int64_t)t + 1];
        const int use_lb = side == 0 ? a > 0 : a < 0;
        f += a * (use_lb ? s->lb[y] : s->ub[y]);
    }
    if (side == 0)
        tell_lb(s, x, ceil_div(f, c[3]));
    else
        tell_ub(s, x, floor_div(f, c[3]));
}

/* ---------------------------------------------------------------------- */
int32_t orc_validate(const orc_model *m)
{
    if (!m || m->nvars < 0 || m->nrows < 0 || m->nreif < 0 || m->ndec < 0)
        return -1;
    if (m->nvars > 0 && (!m->lb0 || !m->ub0))
        return -1;
    if (m->nrows > 0 && (!m->row_ptr || !m->coef || !m->var || !m->rhs))
        return -1;
    if (m->nreif > 0 && !m->reif)
        return -1;
    if (m->ndec > 0 && !m->dec)
        return -1;
    if (m->ncmd < 0 || (m->ncmd > 0 && (!m->cmd || !m->cmd_gptr || !m->cmd_tptr)))
        return -1;
    if (m->objective < -1 || m->objective >= m->nvars)
        return -2;
    for (int32_t k = 0; k < m->ndec; ++k)
        if (m->dec[k] < 0 || m->dec[k] >= m->nvars)
            return -2;
    const int64_t LIM = (int64_t)1 << 31;
    int64_t maxabs_all = 0;
    for (int32_t v = 0; v < m->nvars; ++v) {
        int64_t a = llabs((int64_t)m->lb0[v]), b = llabs((int64_t)m->ub0[v]);
        int64_t mx = a > b ? a : b;
        if (mx > maxabs_all) maxabs_all = mx;
    }
    if (m->nrows > 0 && m->row_ptr[0] != 0)
        return -2;
    char *seen = (char *)calloc(m->nvars > 0 ? (size_t)m->nvars : 1, 1);
    if (!seen)
        return -1;
    int32_t rc = 0;
    for (int32_t r = 0; r < m->nrows && rc == 0; ++r) {
        int32_t a0 = m->row_ptr[r], a1 = m->row_ptr[r + 1];
        if (a1 < a0) { rc = -2; break; }
        int64_t tot = llabs((int64_t)m->rhs[r]);
        for (int32_t t = a0; t < a1; ++t) {
            int32_t x = m->var[t];
            if (x < 0 || x >= m->nvars || m->coef[t] == 0 || seen[x]) { rc = -2; break; }
            seen[x] = 1;
            int64_t a = llabs((int64_t)m->lb0[x]), b = llabs((int64_t)m->ub0[x]);
            tot += llabs((int64_t)m->coef[t]) * (a > b ? a : b);
            if (tot >= LIM) { rc = -3; break; }
        }
        for (int32_t t = a0; t < a1; ++t)
            if (m->var[t] >= 0 && m->var[t] < m->nvars)
                seen[m->var[t]] = 0;
    }
    free(seen);
    if (rc)
        return rc;
    for (int32_t q = 0; q < m->nreif; ++q) {
        const int32_t *it = m->reif + 4 * (int64_t)q;
        for (int k = 0; k < 3; ++k)
            if (it[k] < 0 || it[k] >= m->nvars)
                return -2;
        if (2 * maxabs_all + llabs((int64_t)it[3]) + 1 >= LIM)
            return -3;
    }
    if (m->ncmd > 0 && (m->cmd_gptr[0] != 0 || m->cmd_tptr[0] != 0))
        return -2;
    for (int32_t q = 0; q < m->ncmd; ++q) {
        const int32_t *c = m->cmd + 4 * (int64_t)q;
        if (c[0] < 0 || c[0] >= m->nvars || (c[1] != 0 && c[1] != 1) || c[3] <= 0)
            return -2;
        const int32_t g0 = m->cmd_gptr[q], g1 = m->cmd_gptr[q + 1];
        const int32_t t0 = m->cmd_tptr[q], t1 = m->cmd_tptr[q + 1];
        if (g1 < g0 || t1 < t0 || (g1 > g0 && !m->guard) || (t1 > t0 && !m->cterm))
            return -2;
        for (int32_t g = g0; g < g1; ++g) {
            const int32_t *gd = m->guard + 3 * (int64_t)g;
            if (gd[0] < 0 || gd[0] >= m->nvars || (gd[1] != 0 && gd[1] != 1))
                return -2;
        }
        int64_t tot = llabs((int64_t)c[2]);
        for (int32_t t = t0; t < t1; ++t) {
            const int32_t a = m->cterm[2 * (int64_t)t], y = m->cterm[2 * (int64_t)t + 1];
            if (a == 0 || y < 0 || y >= m->nvars)
                return -2;
            int64_t p = llabs((int64_t)m->lb0[y]), u = llabs((int64_t)m->ub0[y]);
            tot += llabs((int64_t)a) * (p > u ? p : u);
            if (tot >= LIM)
                return -3;
        }
    }
    return 0;
}

static int store_is_failed(const orc_model *m, const store_t *s)
{
    for (int32_t v = 0; v < m->nvars; ++v)
        if (s->lb[v] > s->ub[v])
            return 1;
    return 0;
}

/* SplitMix64, only to draw schedules for the order-independence tests */
static uint64_t sm64(uint64_t *st)
{
    uint64_t z = (*st += 0x9E3779B97F4A7C15ULL);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

static void run_propagator(const orc_model *m, store_t *s, int64_t p)
{
    if (p < m->nrows)
        run_row(m, s, (int32_t)p);
    else if (p < (int64_t)m->nrows + m->nreif)
        run_reif(m, s, (int32_t)(p - m->nrows));
    else
        run_cmd(m, s, (int32_t)(p - m->nrows - m->nreif));
}

/* Jacobi step: every command reads the snapshot (lb0s, ub0s) and joins its
 * tell into the output store (§3, D(P || Q) = D(P) join D(Q)). */
static void jacobi_sweep(const orc_model *m, const int32_t *slb, const int32_t *sub,
                         store_t *out)
{
    /* A command reads only the snapshot; its tell is joined into `out`.
     * To reuse the command code, each command runs on a private copy of the
     * snapshot restricted to the variables it touches, then its result is
     * joined into out. */
    const int32_t V = m->nvars;
    int32_t *tlb = (int32_t *)malloc(sizeof(int32_t) * (size_t)(V > 0 ? V : 1));
    int32_t *tub = (int32_t *)malloc(sizeof(int32_t) * (size_t)(V > 0 ? V : 1));
    memcpy(tlb, slb, sizeof(int32_t) * (size_t)V);
    memcpy(tub, sub, sizeof(int32_t) * (size_t)V);
    store_t t = {tlb, tub, 0, 0};
    for (int32_t r = 0; r < m->nrows; ++r) {
        int32_t a0 = m->row_ptr[r], a1 = m->row_ptr[r + 1];
        for (int32_t k = a0; k < a1; ++k) {
            int32_t x = m->var[k];
            run_row_term(m, &t, r, k);         /* reads snapshot only */
            if (tlb[x] > out->lb[x]) out->lb[x] = tlb[x];
            if (tub[x] < out->ub[x]) out->ub[x] = tub[x];
            tlb[x] = slb[x];
            tub[x] = sub[x];
        }
    }
    for (int32_t q = 0; q < m->nreif; ++q) {
        const int32_t *it = m->reif + 4 * (int64_t)q;
        for (int k = 0; k < REIF_NCMD; ++k) {
            run_reif_cmd(&t, it, k);
            for (int z = 0; z < 3; ++z) {
                int32_t x = it[z];
                if (tlb[x] > out->lb[x]) out->lb[x] = tlb[x];
                if (tub[x] < out->ub[x]) out->ub[x] = tub[x];
                tlb[x] = slb[x];
                tub[x] = sub[x];
            }
        }
    }
    for (int32_t q = 0; q < m->ncmd; ++q) {
        const int32_t x = m->cmd[4 * (int64_t)q];
        run_cmd(m, &t, q);
        if (tlb[x] > out->lb[x]) out->lb[x] = tlb[x];
        if (tub[x] < out->ub[x]) out->ub[x] = tub[x];
        tlb[x] = slb[x];
        tub[x] = sub[x];
    }
    free(tlb);
    free(tub);
}

static int32_t jacobi_step(const orc_model *m, int32_t *lb, int32_t *ub);

int32_t orc_jacobi_step(const orc_model *m, int32_t *lb, int32_t *ub)
{
    int32_t rc = orc_validate(m);
    if (rc)
        return rc;
    if (!lb || !ub)
        return -1;
    return jacobi_step(m, lb, ub);
}

static int32_t jacobi_step(const orc_model *m, int32_t *lb, int32_t *ub)
{
    const int32_t V = m->nvars;
    int32_t *slb = (int32_t *)malloc(sizeof(int32_t) * (size_t)(V > 0 ? V : 1));
    int32_t *sub = (int32_t *)malloc(sizeof(int32_t) * (size_t)(V > 0 ? V : 1));
    memcpy(slb, lb, sizeof(int32_t) * (size_t)V);
    memcpy(sub, ub, sizeof(int32_t) * (size_t)V);
    store_t out = {lb, ub, 0, 0};
    jacobi_sweep(m, slb, sub, &out);
    int changed = memcmp(slb, lb, sizeof(int32_t) * (size_t)V) != 0 ||
                  memcmp(sub, ub, sizeof(int32_t) * (size_t)V) != 0;
    free(slb);
    free(sub);
    if (store_is_failed(m, &out))
        return ORC_FAILED;
    return changed ? 2 : ORC_FIXPOINT;
}

/* One sequential pass: every propagator once, in model order, each tell
 * joined at once (§3, seq P).  Returns ORC_FIXPOINT if nothing changed, 2 if
 * the store changed and is not failed, ORC_FAILED if it became failed. */
int32_t orc_gs_step(const orc_model *m, int32_t *lb, int32_t *ub)
{
    int32_t rc = orc_validate(m);
    if (rc)
        return rc;
    if (!lb || !ub)
        return -1;
    store_t s = {lb, ub, 0, 0};
    if (store_is_failed(m, &s))
        return ORC_FAILED;
    const int64_t P = (int64_t)m->nrows + m->nreif + m->ncmd;
    for (int64_t p = 0; p < P && !s.failed; ++p)
        run_propagator(m, &s, p);
    if (s.failed)
        return ORC_FAILED;
    return s.changed ? 2 : ORC_FIXPOINT;
}

/* propagation loop on an already validated model (the search calls this
 * once per node; orc_propagate validates first) */
int32_t orc_propagate_validated(const orc_model *m, int32_t *lb, int32_t *ub,
                                int32_t sched, uint64_t seed, int64_t *sweeps);

int32_t orc_propagate(const orc_model *m, int32_t *lb, int32_t *ub,
                      int32_t sched, uint64_t seed, int64_t *sweeps)
{
    int32_t rc = orc_validate(m);
    if (rc)
        return rc;
    if (!lb || !ub)
        return -1;
    return orc_propagate_validated(m, lb, ub, sched, seed, sweeps);
}

int32_t orc_propagate_validated(const orc_model *m, int32_t *lb, int32_t *ub,
                                int32_t sched, uint64_t seed, int64_t *sweeps)
{
    store_t s = {lb, ub, 0, 0};
    int64_t nsw = 0;
    if (store_is_failed(m, &s)) {
        if (sweeps) *sweeps = 0;
        return ORC_FAILED;
    }
    const int64_t P = (int64_t)m->nrows + m->nreif + m->ncmd;
    uint64_t rng = seed;

    if (sched == ORC_SCHED_GS || sched == ORC_SCHED_REVERSE || sched == ORC_SCHED_PERM) {
        int64_t *order = (int64_t *)malloc(sizeof(int64_t) * (size_t)(P > 0 ? P : 1));
        for (int64_t p = 0; p < P; ++p)
            order[p] = sched == ORC_SCHED_REVERSE ? P - 1 - p : p;
        do {
            s.changed = 0;
            ++nsw;
            if (sched == ORC_SCHED_PERM)
                for (int64_t p = P - 1; p > 0; --p) {
                    int64_t q = (int64_t)(sm64(&rng) % (uint64_t)(p + 1));
                    int64_t tmp = order[p]; order[p] = order[q]; order[q] = tmp;
                }
            for (int64_t k = 0; k < P && !s.failed; ++k)
                run_propagator(m, &s, order[k]);
        } while (s.changed && !s.failed);
        free(order);
    } else if (sched == ORC_SCHED_JACOBI) {
        for (;;) {
            ++nsw;
            int32_t st = jacobi_step(m, lb, ub);
            if (st == ORC_FAILED) { s.failed = 1; break; }
            if (st == ORC_FIXPOINT) break;
        }
    } else if (sched == ORC_SCHED_SELECT) {
        /* commands: one per row term, REIF_NCMD per reified item, then the
         * model's guarded commands */
        const int64_t T = m->nrows > 0 ? m->row_ptr[m->nrows] : 0;
        const int64_t CR = T + (int64_t)REIF_NCMD * m->nreif;
        const int64_t C = CR + m->ncmd;
        int32_t *term_row = (int32_t *)malloc(sizeof(int32_t) * (size_t)(T > 0 ? T : 1));
        for (int32_t r = 0; r < m->nrows; ++r)
            for (int32_t t = m->row_ptr[r]; t < m->row_ptr[r + 1]; ++t)
                term_row[t] = r;
        for (;;) {
            /* a burst of random selections ... */
            for (int64_t k = 0; k < 2 * C && !s.failed; ++k) {
                int64_t c = C > 0 ? (int64_t)(sm64(&rng) % (uint64_t)C) : 0;
                if (C == 0) break;
                if (c < T)
                    run_row_term(m, &s, term_row[c], (int32_t)c);
                else if (c < CR)
                    run_reif_cmd(&s, m->reif + 4 * ((c - T) / REIF_NCMD),
                                 (int)((c - T) % REIF_NCMD));
                else
                    run_cmd(m, &s, (int32_t)(c - CR));
            }
            if (s.failed) break;
            /* ... then every command once, so that each is selected at least
             * once per round (fairness); stop when that round changes nothing */
            s.changed = 0;
            ++nsw;
            for (int64_t c = 0; c < C && !s.failed; ++c) {
                if (c < T)
                    run_row_term(m, &s, term_row[c], (int32_t)c);
                else if (c < CR)
                    run_reif_cmd(&s, m->reif + 4 * ((c - T) / REIF_NCMD),
                                 (int)((c - T) % REIF_NCMD));
                else
                    run_cmd(m, &s, (int32_t)(c - CR));
            }
            if (s.failed || !s.changed) break;
        }
        free(term_row);
    } else {
        return -1;
    }
    if (sweeps) *sweeps = nsw;
    if (s.failed || store_is_failed(m, &s))
        return ORC_FAILED;
    return ORC_FIXPOINT;
}
