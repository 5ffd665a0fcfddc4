/*
 * CPU oracle for PCCP propagation and propagate-and-search.
 *
 * TEST INFRASTRUCTURE ONLY.  This library is a plain, sequential, obviously
 * correct statement of what the solver computes; it exists so that tests, the
 * smoke check and the benchmark's CPU-baseline leg can check the HIP solver
 * against it.  The product (libpccp and its Python binding) never links,
 * loads or calls it, and it shares no source with the product.
 *
 * Paper: P. Talbot, F. Pinel, P. Bouvry, "A Variant of Concurrent Constraint
 * Programming on GPU", AAAI 2022 (arXiv 2207.12116).
 *
 * What is computed (and where it is defined):
 *   - Store: one interval (lb, ub) of the lattice IZ = ZInc x ZDec per
 *     variable (§2, interval lattice); a store with an empty interval is the
 *     failed store (top), detected at once (§5, fixed point loop: failure is
 *     a fixed point on top).
 *   - Linear row  sum_t a_t * x_t <= c: the bound tell of §2 (compilation of
 *     x + y <= c), generalised to any nonzero integer coefficients with
 *     rounding toward -inf / +inf.  The resource sums of §2 are such rows.
 *   - Reified overlap  b <=> (si <= sj and sj < si + d): the four guarded
 *     processes of §2 (compilation of phi <=> psi), with the entailment tests
 *     of §2 extended to conjunction and negation, and disjunction propagated
 *     by the usual "one disjunct disentailed" rule (the paper gives no
 *     compilation of a disjunction or of negated entailment).
 *   - Guarded command  {g_1..g_n} => x <- f(y_1..y_m) (§3, guarded normal
 *     form; §2, ask and tell statements): when every guard is entailed,
 *     join f into one bound of x.  Guards are entailment tests of a bound
 *     against a constant; f is an affine form over the bounds that make it
 *     monotone, divided and rounded toward the side that keeps it sound.
 *   - propagate: the least fixed point above a store (§3, Theorem 2), computed
 *     by the sequential composition of all guarded commands repeated until
 *     nothing changes (§3, Proposition 3: seq P has the same fixed point).
 *     Jacobi, random-permutation, random-selection and reversed schedules are
 *     provided for the order-independence tests (§3, fairness and chaotic
 *     iterations; Theorem 6).
 *   - solve: depth-first propagate-and-search (§1), splitting a node into the
 *     complementary subproblems x = lb(x) and x >= lb(x) + 1, first-fail
 *     variable choice (smallest width, ties to the earliest decision
 *     variable), and branch-and-bound on the objective for minimisation.
 *
 * Error codes: 0 OK; -1 invalid argument; -2 malformed model (index out of
 * range, duplicate variable in a row, zero coefficient); -3 int32 overflow
 * risk (sum |a| * max(|lb|,|ub|) + |c| >= 2^31).
 */
#ifndef PCCP_ORACLE_H
#define PCCP_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t nvars;
    const int32_t *lb0, *ub0;          /* initial box, nvars each            */
    int32_t nrows;
    const int32_t *row_ptr;            /* nrows + 1                          */
    const int32_t *coef, *var;         /* row_ptr[nrows] terms               */
    const int32_t *rhs;                /* nrows                              */
    int32_t nreif;
    const int32_t *reif;               /* 4 per item: b, si, sj, d           */
    int32_t ndec;
    const int32_t *dec;                /* decision variables, tie-break order*/
    int32_t objective;                 /* -1 if none                          */
    /* guarded commands (§3, guarded normal form):
     *   {g_1, ..., g_n} => x <- f,  f = k + sum_t a_t * y_t,
     * cmd: 4 per command: x, side (0: lb(x) >= ceil(f / div), 1: ub(x) <=
     * floor(f / div)), k, div (> 0);  guards of command q:
     * guard[3*g .. 3*g+2] for g in [cmd_gptr[q], cmd_gptr[q+1]): var, side
     * (0: entailed(var >= c) = lb(var) >= c, 1: entailed(var <= c) =
     * ub(var) <= c), c;  terms of command q: cterm[2*t], cterm[2*t+1] =
     * a_t, y_t for t in [cmd_tptr[q], cmd_tptr[q+1]).                      */
    int32_t ncmd;
    const int32_t *cmd;
    const int32_t *cmd_gptr;
    const int32_t *guard;
    const int32_t *cmd_tptr;
    const int32_t *cterm;
} orc_model;

enum { ORC_FIXPOINT = 0, ORC_FAILED = 1 };

/* schedules of the propagation loop (all must reach the same result) */
enum {
    ORC_SCHED_GS = 0,       /* model order, tells applied at once           */
    ORC_SCHED_JACOBI = 1,   /* every tell of a sweep reads the same snapshot */
    ORC_SCHED_PERM = 2,     /* a fresh random propagator order every sweep  */
    ORC_SCHED_SELECT = 3,   /* random single guarded commands, fair         */
    ORC_SCHED_REVERSE = 4   /* reversed model order                         */
};

enum { ORC_ENUMERATE = 0, ORC_MINIMIZE = 1 };
enum { ORC_FIRST_FAIL = 0, ORC_INPUT_ORDER = 1, ORC_EXPERT = 2 /* learn.c */,
       ORC_MLP = 3 /* network scores, see orc_set_mlp_params */ };
void orc_set_mlp_params(const double *p);
enum {
    ORC_OUT_ALL = 0,        /* ENUMERATE: search tree exhausted             */
    ORC_OUT_OPTIMAL = 1,    /* MINIMIZE: best solution proven optimal       */
    ORC_OUT_UNSAT = 2,      /* MINIMIZE: no solution                        */
    ORC_OUT_LIMIT = 3       /* node limit reached                           */
};

typedef struct {
    int64_t nodes;          /* propagate calls, including failed ones/leaves */
    int64_t fails;
    int64_t solutions;
    int64_t max_depth;
    int64_t sweeps;         /* sweeps of the propagation loop, summed        */
    int32_t best;           /* MINIMIZE: best objective (INT32_MAX if none) */
    int32_t outcome;
    uint64_t sol_hash;      /* order-independent hash of the solution set   */
} orc_stats;

int32_t orc_validate(const orc_model *m);

/* Fixed point above (lb, ub), in place.  Returns ORC_FIXPOINT or ORC_FAILED,
 * or a negative error.  On ORC_FAILED the contents of lb/ub are unspecified. */
int32_t orc_propagate(const orc_model *m, int32_t *lb, int32_t *ub,
                      int32_t sched, uint64_t seed, int64_t *sweeps);

/* One parallel (Jacobi) application of every guarded command:
 * s := s join tells(s).  Returns ORC_FIXPOINT if s is unchanged,
 * 2 if s changed and is not failed, ORC_FAILED if s became failed. */
int32_t orc_jacobi_step(const orc_model *m, int32_t *lb, int32_t *ub);

/* One sequential (Gauss-Seidel) pass over every propagator in model order;
 * same return convention as orc_jacobi_step. */
int32_t orc_gs_step(const orc_model *m, int32_t *lb, int32_t *ub);

/* Depth-first search.  sol_buf (may be NULL) receives up to sol_cap
 * solutions of ndec values each, in discovery order; best_assign (may be
 * NULL) receives the ndec decision values of the best solution. */
int32_t orc_solve(const orc_model *m, int32_t mode, int32_t branching,
                  int64_t node_limit, int32_t *sol_buf, int64_t sol_cap,
                  int32_t *best_assign, orc_stats *st);

/* Hash of one solution (FNV-1a 64 over the little-endian bytes, finalised
 * by MurmurHash3's fmix64); the solution-set hash is the wrapping sum. */
uint64_t orc_solution_hash(const int32_t *vals, int32_t n);

/* Timing harness (timing.c): orc_solve on n independent instances, one
 * POSIX thread per host core (threads), each taking the next instance.
 * Per instance: nodes, seconds (CLOCK_MONOTONIC), outcome and best; wall_s
 * is the whole set's time.  Returns 0, or the first negative error of
 * orc_solve (the other instances still run). */
int32_t orc_solve_timed(const orc_model *const *models, int32_t n, int32_t mode,
                        int32_t branching, int64_t node_limit, int32_t threads,
                        int64_t *nodes, double *secs, int32_t *outcome, int32_t *best,
                        double *wall_s);

/* ---- brute force (independent of the propagation code) ---------------- */

/* All integer points of the initial box satisfying every linear row and
 * every reified item.  Counts them, hashes their decision-variable values,
 * and copies up to cap of them (ndec values each) to out. */
int64_t orc_brute_points(const orc_model *m, int32_t *out, int64_t cap,
                         uint64_t *hash);

/* Minimum makespan of a raw RCPSP <T, P, R> by enumerating start times in
 * [0, h - d_i] and checking precedences and the per-instant resource
 * profile directly.  Returns -1 if no schedule exists.  best_s (may be NULL)
 * receives one optimal schedule. */
int32_t orc_brute_rcpsp(int32_t n, const int32_t *dur, int32_t nedges,
                        const int32_t *edges, int32_t nres, const int32_t *dem,
                        const int32_t *cap, int32_t h, int32_t *best_s);

/* Check a schedule against the raw RCPSP data, instant by instant.
 * Returns 1 if feasible, 0 otherwise; *makespan gets max(s_i + d_i). */
int32_t orc_check_schedule(int32_t n, const int32_t *dur, int32_t nedges,
                           const int32_t *edges, int32_t nres,
                           const int32_t *dem, const int32_t *cap,
                           const int32_t *s, int32_t *makespan);

/* ---- learned branching (learn.c) ----------------------------------- */

/* Features of every decision variable in the store (lb, ub): 6 doubles per
 * decision variable, in decision-list order (definitions in learn.c). */
int32_t orc_features(const orc_model *m, const int32_t *lb, const int32_t *ub, double *out);

/* Scores of ncand candidates (6 features each) under parameters p (513). */
int32_t orc_mlp_forward(const double *p, const double *x, int64_t ncand, double *scores);

/* Mean per-node cross-entropy between targets t (per candidate, summing to
 * 1 over each node) and the softmax of the scores; gradient (513 values). */
int32_t orc_mlp_loss_grad(const double *p, const double *x, const int32_t *node_off,
                          const double *t, int32_t nnodes, double *loss, double *g);

/* The network's branching choice at a propagated store: the decision-list
 * position of the unfixed candidate with the largest score under p (ties to
 * the earliest), or -1 if every decision variable is fixed. */
int32_t orc_mlp_choice(const orc_model *m, const double *p, const int32_t *lb, const int32_t *ub);

/* One Adam step in place (beta1 0.9, beta2 0.999, eps 1e-8; step >= 1). */
int32_t orc_adam_step(double *p, const double *g, double *m, double *v, int32_t n, double lr,
                      int32_t step);

/* Search traces with expert labels (see learn.c). */
int64_t orc_trace(const orc_model *m, int32_t mode, int64_t node_limit, float *feat,
                  double *score, int32_t *cand, int32_t *off, int32_t *label, int64_t cap_nodes,
                  int64_t cap_cand, int64_t *ncand);

/* ---- floating-point interval stores (fprop.c) ----------------------- */

/* A model over float32 interval variables (§2: FInc x FDec, IEEE total
 * order) with linear rows sum_t coef[t] * x_var[t] <= rhs over the reals;
 * propagation rounds outward (fprop.c).  Initial bounds must be finite. */
typedef struct {
    int32_t nvars;
    const float *lb0, *ub0;
    int32_t nrows;
    const int32_t *row_ptr;            /* nrows + 1                          */
    const float *coef;                 /* row_ptr[nrows]                     */
    const int32_t *var;
    const float *rhs;                  /* nrows                              */
} orc_fmodel;

/* 0, or -1 (bad arguments) / -2 (non-finite bound or coefficient, zero
 * coefficient, index out of range, variable repeated in a row). */
int32_t orc_fvalidate(const orc_fmodel *m);

/* Least fixed point above (lb, ub), in place (zeros made canonical first:
 * -0 for lower bounds, +0 for upper bounds).  Schedules: ORC_SCHED_GS,
 * _JACOBI, _PERM (seeded), _REVERSE.  ORC_FIXPOINT or ORC_FAILED. */
int32_t orc_fpropagate(const orc_fmodel *m, float *lb, float *ub, int32_t sched, uint64_t seed,
                       int64_t *sweeps);

/* One Jacobi step: ORC_FIXPOINT if nothing changed, 2 if the store changed
 * and is not failed, ORC_FAILED. */
int32_t orc_fjacobi_step(const orc_fmodel *m, float *lb, float *ub);

/* 1 if a and b (n floats) are bit-identical. */
int32_t orc_fsame(int32_t n, const float *a, const float *b);

#ifdef __cplusplus
}
#endif
#endif
