/*
 * CPU oracle: depth-first propagate-and-search.  TEST INFRASTRUCTURE ONLY
 * (see oracle.h); never linked into the product.
 *
 * Propagate-and-search (§1): propagate a node to its fixed point; if it
 * failed, backtrack; if every decision variable is fixed, it is a solution;
 * otherwise split it into two complementary subproblems and search both.
 *   - split on variable v with value l = lb(v): left child ub(v) := l
 *     (v = l), right child lb(v) := l + 1; left first.
 *   - v: first-fail (smallest ub - lb among unfixed decision variables, ties
 *     to the earliest in the decision list) or input order (the earliest
 *     unfixed one).  The paper states only that the same strategy was used
 *     for both solvers it compares (§5, Evaluation).
 *   - minimisation by branch-and-bound: every node, before propagating, joins
 *     ub(objective) <= best - 1; a solution's value is lb(objective).
 * A node is one propagate call (failed nodes and solutions included).
 * This implementation keeps a private copy of the store per node; the GPU
 * solver recomputes from a subproblem root instead (§5, Turbo).  Both give
 * the same node stores because propagation is a closure operator
 * (§3, Theorem 2).
 */
#include "oracle.h"

#include <stdint.h>
#include <stdlib.h>
#include <string.h>

int32_t orc_propagate_validated(const orc_model *m, int32_t *lb, int32_t *ub,
                                int32_t sched, uint64_t seed, int64_t *sweeps);

/* FNV-1a 64-bit over the little-endian bytes of the values, finalised with
 * MurmurHash3's fmix64. */
uint64_t orc_solution_hash(const int32_t *vals, int32_t n)
{
    uint64_t h = 0xcbf29ce484222325ULL;
    for (int32_t i = 0; i < n; ++i) {
        uint32_t v = (uint32_t)vals[i];
        for (int k = 0; k < 4; ++k) {
            h ^= (v >> (8 * k)) & 0xffu;
            h *= 0x100000001b3ULL;
        }
    }
    h ^= h >> 33;
    h *= 0xff51afd7ed558ccdULL;
    h ^= h >> 33;
    h *= 0xc4ceb9fe1a85ec53ULL;
    h ^= h >> 33;
    return h;
}

typedef struct {
    const orc_model *m;
    int32_t mode, branching;
    int64_t node_limit;
    int32_t *sol_buf;
    int64_t sol_cap;
    int32_t *best_assign;
    int32_t *vals;          /* scratch: decision values of a solution */
    orc_stats *st;
    int hit_limit;
} ctx_t;

int32_t orc_expert_choice(const orc_model *m, const int32_t *lb, const int32_t *ub);
int32_t orc_mlp_choice(const orc_model *m, const double *p, const int32_t *lb, const int32_t *ub);
static const double *g_mlp_params = NULL;  /* set by orc_set_mlp_params */

/* Parameters (513 doubles, see learn.c) used by ORC_MLP branching; the
 * caller keeps them alive during the searches.  Not thread-safe. */
void orc_set_mlp_params(const double *p) { g_mlp_params = p; }

/* index into m->dec of the branching variable, or -1 if all are fixed */
static int32_t choose(const ctx_t *c, const int32_t *lb, const int32_t *ub)
{
    const orc_model *m = c->m;
    if (c->branching == ORC_EXPERT)
        return orc_expert_choice(m, lb, ub);
    if (c->branching == ORC_MLP)
        return orc_mlp_choice(m, g_mlp_params, lb, ub);
    int32_t pick = -1;
    int64_t best_w = 0;
    for (int32_t k = 0; k < m->ndec; ++k) {
        int32_t v = m->dec[k];
        int64_t w = (int64_t)ub[v] - lb[v];
        if (w <= 0)
            continue;
        if (c->branching == ORC_INPUT_ORDER)
            return k;
        if (pick < 0 || w < best_w) {
            pick = k;
            best_w = w;
        }
    }
    return pick;
}

static void dfs(ctx_t *c, const int32_t *plb, const int32_t *pub, int64_t depth)
{
    const orc_model *m = c->m;
    orc_stats *st = c->st;
    if (c->hit_limit)
        return;
    if (c->node_limit > 0 && st->nodes >= c->node_limit) {
        c->hit_limit = 1;
        return;
    }
    const size_t bytes = sizeof(int32_t) * (size_t)(m->nvars > 0 ? m->nvars : 1);
    int32_t *lb = (int32_t *)malloc(bytes), *ub = (int32_t *)malloc(bytes);
    memcpy(lb, plb, sizeof(int32_t) * (size_t)m->nvars);
    memcpy(ub, pub, sizeof(int32_t) * (size_t)m->nvars);

    st->nodes += 1;
    if (depth > st->max_depth)
        st->max_depth = depth;
    if (c->mode == ORC_MINIMIZE && st->best != INT32_MAX &&
        (int64_t)st->best - 1 < ub[m->objective])
        ub[m->objective] = st->best - 1;

    int64_t sw = 0;
    int32_t status = orc_propagate_validated(m, lb, ub, ORC_SCHED_GS, 0, &sw);
    st->sweeps += sw;
    if (status != ORC_FIXPOINT) {
        st->fails += 1;
        goto done;
    }
    int32_t k = choose(c, lb, ub);
    if (k < 0) {                            /* every decision variable fixed */
        for (int32_t q = 0; q < m->ndec; ++q)
            c->vals[q] = lb[m->dec[q]];
        if (c->mode == ORC_ENUMERATE) {
            if (c->sol_buf && st->solutions < c->sol_cap)
                memcpy(c->sol_buf + st->solutions * (int64_t)m->ndec, c->vals,
                       sizeof(int32_t) * (size_t)m->ndec);
            st->sol_hash += orc_solution_hash(c->vals, m->ndec);
        } else {
            int32_t obj = lb[m->objective];
            if (obj < st->best) {
                st->best = obj;
                if (c->best_assign)
                    memcpy(c->best_assign, c->vals, sizeof(int32_t) * (size_t)m->ndec);
            }
        }
        st->solutions += 1;
        goto done;
    }
    {
        int32_t v = m->dec[k];
        int32_t val = lb[v];
        int32_t keep_ub = ub[v];
        ub[v] = val;                        /* left: v = lb(v) */
        dfs(c, lb, ub, depth + 1);
        ub[v] = keep_ub;
        lb[v] = val + 1;                    /* right: v >= lb(v) + 1 */
        dfs(c, lb, ub, depth + 1);
    }
done:
    free(lb);
    free(ub);
}

int32_t orc_solve(const orc_model *m, int32_t mode, int32_t branching,
                  int64_t node_limit, int32_t *sol_buf, int64_t sol_cap,
                  int32_t *best_assign, orc_stats *st)
{
    int32_t rc = orc_validate(m);
    if (rc)
        return rc;
    if (!st || (mode != ORC_ENUMERATE && mode != ORC_MINIMIZE) ||
        (branching != ORC_FIRST_FAIL && branching != ORC_INPUT_ORDER && branching != ORC_EXPERT &&
         branching != ORC_MLP) || (branching == ORC_MLP && !g_mlp_params))
        return -1;
    if (mode == ORC_MINIMIZE && m->objective < 0)
        return -1;
    memset(st, 0, sizeof(*st));
    st->best = INT32_MAX;
    ctx_t c;
    memset(&c, 0, sizeof(c));
    c.m = m;
    c.mode = mode;
    c.branching = branching;
    c.node_limit = node_limit;
    c.sol_buf = sol_buf;
    c.sol_cap = sol_buf ? sol_cap : 0;
    c.best_assign = best_assign;
    c.st = st;
    c.vals = (int32_t *)malloc(sizeof(int32_t) * (size_t)(m->ndec > 0 ? m->ndec : 1));
    dfs(&c, m->lb0, m->ub0, 0);
    free(c.vals);
    if (c.hit_limit)
        st->outcome = ORC_OUT_LIMIT;
    else if (mode == ORC_ENUMERATE)
        st->outcome = ORC_OUT_ALL;
    else
        st->outcome = st->best == INT32_MAX ? ORC_OUT_UNSAT : ORC_OUT_OPTIMAL;
    return 0;
}
