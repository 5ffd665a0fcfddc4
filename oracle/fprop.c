/*
 * CPU oracle: propagation over floating-point interval stores.  TEST
 * INFRASTRUCTURE ONLY (see oracle.h); never linked into the product.
 *
 * The store holds one interval (lb, ub) of float32 bounds per variable: lb
 * in the lattice FInc and ub in FDec of §2 (increasing / decreasing
 * floating-point numbers), ordered by the IEEE 754-2019 total order as the
 * footnote of §2 suggests.  The only values where that order differs from
 * the numeric one among finite bounds are the two zeros (-0 < +0); bounds
 * are kept canonical so that the two orders agree on every comparison the
 * propagation makes: a lower bound that is zero is -0 and an upper bound
 * that is zero is +0 (the weaker of the two in each lattice).  A store is
 * failed when some lb > ub.
 *
 * Constraint: the linear row sum_t a_t x_t <= c over the reals, with float32
 * coefficients and right-hand side.  Its tells are those of the integer row
 * (§2: x + y <= c tells ub(x) <= c - lb(y); generalised to any
 * coefficients), computed with outward rounding so that no real solution is
 * lost (§6: intervals of reals are approximated by intervals of floats):
 *   m_u  = the least value of a_u x_u over the box, rounded down
 *          (a_u lb(x_u) if a_u > 0, else a_u ub(x_u))
 *   S_t  = the sum of m_u over the other terms u != t, in term order, each
 *          addition rounded down, starting from +0
 *   num  = c - S_t rounded up
 *   a_t > 0:  ub(x_t) <- ub(x_t) meet (num / a_t rounded up)
 *   a_t < 0:  lb(x_t) <- lb(x_t) join (num / a_t rounded down)
 * Every step is monotone in the store (rounding is monotone), so each tell
 * is a monotone function and the least fixed point above a store is unique
 * and reached by any fair schedule (§3, Theorem 2); the schedules below
 * must agree bit for bit.
 *
 * Rounding: each operation runs in its own rounding mode set with
 * fesetround, on operands read through volatile objects after the mode is
 * set, so that no operation is moved across a mode change.
 */
#include "oracle.h"

#include <fenv.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

/* gcc ignores the FENV_ACCESS pragma; the library is built with
 * -frounding-math, and the volatile operands below keep every operation
 * between its mode changes */

static float rd_mul(float a, float b)
{
    fesetround(FE_DOWNWARD);
    volatile float x = a, y = b;
    volatile float r = x * y;
    fesetround(FE_TONEAREST);
    return r;
}
static float rd_add(float a, float b)
{
    fesetround(FE_DOWNWARD);
    volatile float x = a, y = b;
    volatile float r = x + y;
    fesetround(FE_TONEAREST);
    return r;
}
static float ru_sub(float a, float b)
{
    fesetround(FE_UPWARD);
    volatile float x = a, y = b;
    volatile float r = x - y;
    fesetround(FE_TONEAREST);
    return r;
}
static float rd_div(float a, float b)
{
    fesetround(FE_DOWNWARD);
    volatile float x = a, y = b;
    volatile float r = x / y;
    fesetround(FE_TONEAREST);
    return r;
}
static float ru_div(float a, float b)
{
    fesetround(FE_UPWARD);
    volatile float x = a, y = b;
    volatile float r = x / y;
    fesetround(FE_TONEAREST);
    return r;
}

/* canonical zeros: -0 for a lower bound, +0 for an upper bound */
static float canon_lb(float v) { return v == 0.0f ? -0.0f : v; }
static float canon_ub(float v) { return v == 0.0f ? 0.0f : v; }

static int same_bits(float a, float b) { return memcmp(&a, &b, sizeof(float)) == 0; }

int32_t orc_fvalidate(const orc_fmodel *m)
{
    if (!m || m->nvars < 0 || m->nrows < 0) return -1;
    if (m->nvars > 0 && (!m->lb0 || !m->ub0)) return -1;
    if (m->nrows > 0 && (!m->row_ptr || !m->coef || !m->var || !m->rhs)) return -1;
    for (int32_t v = 0; v < m->nvars; ++v)
        if (!isfinite(m->lb0[v]) || !isfinite(m->ub0[v])) return -2;
    if (m->nrows > 0 && m->row_ptr[0] != 0) return -2;
    char *seen = (char *)calloc((size_t)(m->nvars > 0 ? m->nvars : 1), 1);
    if (!seen) return -1;
    int32_t rc = 0;
    for (int32_t r = 0; r < m->nrows && rc == 0; ++r) {
        const int32_t a0 = m->row_ptr[r], a1 = m->row_ptr[r + 1];
        if (a1 <= a0 || !isfinite(m->rhs[r])) { rc = -2; break; }
        for (int32_t t = a0; t < a1; ++t) {
            const int32_t x = m->var[t];
            if (x < 0 || x >= m->nvars || !isfinite(m->coef[t]) || m->coef[t] == 0.0f || seen[x]) {
                rc = -2;
                break;
            }
            seen[x] = 1;
        }
        for (int32_t t = a0; t < a1; ++t)
            if (m->var[t] >= 0 && m->var[t] < m->nvars) seen[m->var[t]] = 0;
    }
    free(seen);
    return rc;
}

/* The tell of term t of row r read from (lb, ub): the value for x_t and
 * whether it is an upper bound (1) or a lower bound (0). */
static int ftell(const orc_fmodel *m, const float *lb, const float *ub, int32_t r, int32_t t,
                 float *val)
{
    float s = 0.0f;
    for (int32_t u = m->row_ptr[r]; u < m->row_ptr[r + 1]; ++u) {
        if (u == t) continue;
        const float a = m->coef[u];
        const int32_t y = m->var[u];
        s = rd_add(s, rd_mul(a, a > 0.0f ? lb[y] : ub[y]));
    }
    const float num = ru_sub(m->rhs[r], s);
    const float a = m->coef[t];
    if (a > 0.0f) {
        *val = canon_ub(ru_div(num, a));
        return 1;
    }
    *val = canon_lb(rd_div(num, a));
    return 0;
}

/* join the tell into the store; 1 if the store changed */
static int fapply(float *lb, float *ub, int32_t x, int is_ub, float v)
{
    if (is_ub) {
        if (v < ub[x]) { ub[x] = v; return 1; }
    } else {
        if (v > lb[x]) { lb[x] = v; return 1; }
    }
    return 0;
}

static int ffailed(const orc_fmodel *m, const float *lb, const float *ub)
{
    for (int32_t v = 0; v < m->nvars; ++v)
        if (lb[v] > ub[v]) return 1;
    return 0;
}

static uint64_t fsm64(uint64_t *s)
{
    uint64_t z = (*s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

int32_t orc_fpropagate(const orc_fmodel *m, float *lb, float *ub, int32_t sched, uint64_t seed,
                       int64_t *sweeps)
{
    int32_t rc = orc_fvalidate(m);
    if (rc < 0) return rc;
    if ((m->nvars > 0 && (!lb || !ub)) || sched < ORC_SCHED_GS || sched > ORC_SCHED_REVERSE ||
        sched == ORC_SCHED_SELECT)
        return -1;
    for (int32_t v = 0; v < m->nvars; ++v) {
        if (isnan(lb[v]) || isnan(ub[v])) return -1;
        lb[v] = canon_lb(lb[v]);
        ub[v] = canon_ub(ub[v]);
    }
    const int32_t T = m->nrows > 0 ? m->row_ptr[m->nrows] : 0;
    /* term index -> row */
    int32_t *row_of = (int32_t *)malloc(sizeof(int32_t) * (size_t)(T > 0 ? T : 1));
    int32_t *order = (int32_t *)malloc(sizeof(int32_t) * (size_t)(T > 0 ? T : 1));
    float *vals = (float *)malloc(sizeof(float) * (size_t)(T > 0 ? T : 1));
    int *kinds = (int *)malloc(sizeof(int) * (size_t)(T > 0 ? T : 1));
    if (!row_of || !order || !vals || !kinds) {
        free(row_of); free(order); free(vals); free(kinds);
        return -1;
    }
    for (int32_t r = 0; r < m->nrows; ++r)
        for (int32_t t = m->row_ptr[r]; t < m->row_ptr[r + 1]; ++t) row_of[t] = r;
    for (int32_t t = 0; t < T; ++t) order[t] = t;
    uint64_t rng = seed;
    int64_t nsw = 0;
    int32_t status = ORC_FIXPOINT;
    if (ffailed(m, lb, ub)) status = ORC_FAILED;
    while (status == ORC_FIXPOINT) {
        ++nsw;
        int changed = 0;
        if (sched == ORC_SCHED_JACOBI) {
            /* every tell reads the same snapshot, then all are joined */
            for (int32_t t = 0; t < T; ++t) kinds[t] = ftell(m, lb, ub, row_of[t], t, &vals[t]);
            for (int32_t t = 0; t < T; ++t) changed |= fapply(lb, ub, m->var[t], kinds[t], vals[t]);
        } else {
            if (sched == ORC_SCHED_PERM)
                for (int32_t i = T - 1; i > 0; --i) {
                    const int32_t j = (int32_t)(fsm64(&rng) % (uint64_t)(i + 1));
                    const int32_t tmp = order[i];
                    order[i] = order[j];
                    order[j] = tmp;
                }
            for (int32_t i = 0; i < T; ++i) {
                const int32_t t = sched == ORC_SCHED_REVERSE ? T - 1 - i : order[i];
                float v;
                const int k = ftell(m, lb, ub, row_of[t], t, &v);
                changed |= fapply(lb, ub, m->var[t], k, v);
                if (lb[m->var[t]] > ub[m->var[t]]) break;
            }
        }
        if (ffailed(m, lb, ub)) status = ORC_FAILED;
        else if (!changed) break;
    }
    free(row_of); free(order); free(vals); free(kinds);
    if (sweeps) *sweeps = nsw;
    return status;
}

/* One Jacobi step (every tell from the same snapshot, then joined):
 * ORC_FIXPOINT if unchanged, 2 if changed and not failed, ORC_FAILED. */
int32_t orc_fjacobi_step(const orc_fmodel *m, float *lb, float *ub)
{
    int32_t rc = orc_fvalidate(m);
    if (rc < 0) return rc;
    const int32_t T = m->nrows > 0 ? m->row_ptr[m->nrows] : 0;
    float *vals = (float *)malloc(sizeof(float) * (size_t)(T > 0 ? T : 1));
    int *kinds = (int *)malloc(sizeof(int) * (size_t)(T > 0 ? T : 1));
    if (!vals || !kinds) { free(vals); free(kinds); return -1; }
    for (int32_t r = 0; r < m->nrows; ++r)
        for (int32_t t = m->row_ptr[r]; t < m->row_ptr[r + 1]; ++t)
            kinds[t] = ftell(m, lb, ub, r, t, &vals[t]);
    int changed = 0;
    for (int32_t t = 0; t < T; ++t) changed |= fapply(lb, ub, m->var[t], kinds[t], vals[t]);
    free(vals); free(kinds);
    if (ffailed(m, lb, ub)) return ORC_FAILED;
    return changed ? 2 : ORC_FIXPOINT;
}

/* 1 if the two stores are bit-identical */
int32_t orc_fsame(int32_t n, const float *a, const float *b)
{
    for (int32_t i = 0; i < n; ++i)
        if (!same_bits(a[i], b[i])) return 0;
    return 1;
}
