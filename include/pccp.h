/*
 * libpccp - lock-free parallel constraint propagation and propagate-and-search
 * on one AMD Instinct MI355X (gfx950).
 *
 * Method: P. Talbot, F. Pinel, P. Bouvry, "A Variant of Concurrent Constraint
 * Programming on GPU", AAAI 2022 (arXiv 2207.12116).
 *
 * Vocabulary.
 *   variable   an integer interval (lb, ub) of the lattice IZ = ZInc x ZDec
 *              (§2); values are int32.  A store is one interval per variable
 *              (§3: names erased to indices).  A store with lb > ub somewhere
 *              is the failed store (top).
 *   propagator the process compiling one constraint (§2, [[.]]).  Two
 *              constraint forms are supported:
 *                linear   sum_t a_t x_t <= c       (§2, [[x + y <= c]] and the
 *                                                   resource sums)
 *                reified  b <=> (si <= sj and sj < si + d)
 *                                                  (§2, [[phi <=> psi]] as used
 *                                                   by the RCPSP model)
 *   fixed point the least store above a given store at which no propagator
 *              tightens a bound (§3, Theorem 2); it is unique and does not
 *              depend on the order in which propagators run (§3, Theorem 6;
 *              §4, Theorems 8 and 9).
 *   search     depth-first propagate-and-search (§1) over the decision
 *              variables: a node's store is propagated; a failed node is
 *              pruned; a node whose decision variables are all fixed is a
 *              solution; otherwise it splits into x = lb(x) and x >= lb(x)+1
 *              on the variable chosen by the branching rule.  Minimisation is
 *              branch-and-bound: every node joins ub(objective) <= best - 1.
 *
 * Conventions.
 *   - Every function returns int32_t: PCCP_OK (0) or a negative error code.
 *     Solver outcomes (fixed point / failed, optimal / unsat / limit) are
 *     returned through out-parameters, not as errors.
 *   - pccp_last_error() returns a thread-local description of the last
 *     error of the calling thread.  No C++ exception crosses this interface.
 *   - Handles are opaque and owned by the library (create / destroy).
 *     Host arrays passed in are copied during the call; output arrays are
 *     owned by the caller and sized as documented.  Device pointers passed
 *     in are owned by the caller; the library never frees them.
 *   - A solver is bound to the HIP device that is current when it is created
 *     and to the HIP stream given then (0 = the null stream).  All device
 *     work is enqueued on that stream; calls that return host data
 *     synchronise that stream only.
 *   - Limits: at most 65535 variables per model, and the store (8 bytes per
 *     variable) must fit in one workgroup's LDS; linear coefficients and
 *     reified offsets d must fit in int16; every row must satisfy
 *     sum |a_t| * max(|lb|, |ub|) + |c| < 2^30 so that int32 arithmetic
 *     cannot overflow.  Violations are reported at solver creation.
 */
#ifndef PCCP_H
#define PCCP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes ------------------------------------------------------- */
#define PCCP_OK 0
#define PCCP_E_INVALID_ARG (-1)  /* null pointer, negative size, bad enum    */
#define PCCP_E_MODEL (-2)        /* index out of range, duplicate variable in
                                    a row, zero coefficient, empty row       */
#define PCCP_E_OVERFLOW (-3)     /* int32 overflow possible (see Limits)     */
#define PCCP_E_NOMEM (-4)        /* host or device allocation failed         */
#define PCCP_E_DEVICE (-5)       /* a HIP call failed (text kept)            */
#define PCCP_E_LDS_CAPACITY (-6) /* the store does not fit in LDS            */
#define PCCP_E_STATE (-7)        /* call out of order (e.g. no result yet)   */
#define PCCP_E_UNSUPPORTED (-8)  /* value outside the packed layouts         */
#define PCCP_E_DEPTH (-9)        /* a search path exceeded max_depth          */

/* ---- outcomes ---------------------------------------------------------- */
#define PCCP_FIXPOINT 0          /* propagate: the least fixed point reached */
#define PCCP_FAILED 1            /* propagate: the fixed point is failed     */

#define PCCP_ENUMERATE 0         /* search mode: all solutions               */
#define PCCP_MINIMIZE 1          /* search mode: minimise the objective      */

#define PCCP_OUT_ALL 0           /* ENUMERATE finished: every solution found */
#define PCCP_OUT_OPTIMAL 1       /* MINIMIZE finished: best is optimal       */
#define PCCP_OUT_UNSAT 2         /* MINIMIZE finished: no solution           */
#define PCCP_OUT_LIMIT 3         /* node or time limit reached               */
#define PCCP_OUT_CANCELLED 4     /* the cancel word was set                  */

#define PCCP_BRANCH_FIRST_FAIL 0 /* smallest ub - lb, ties to the earliest
                                    decision variable                        */
#define PCCP_BRANCH_INPUT_ORDER 1/* the earliest unfixed decision variable   */
#define PCCP_BRANCH_MLP 2        /* learned scores (pccp_mlp_*)              */

typedef struct pccp_model pccp_model;
typedef struct pccp_solver pccp_solver;
typedef struct pccp_fmodel pccp_fmodel;
typedef struct pccp_fsolver pccp_fsolver;

/* ---- model building (host) -------------------------------------------- */
/* §2 (modelling layer): a model declares interval variables and constraints;
 * the library compiles each constraint to its propagator. */

/* Create an empty model.  *out receives the handle. */
int32_t pccp_model_create(pccp_model **out);
int32_t pccp_model_destroy(pccp_model *m);

/* Append n variables with initial intervals [lb[i], ub[i]] (§2, the tell
 * x <- (l, u) that initialises a variable).  lb > ub is allowed: the model's
 * root store is then failed.  *first_id (may be NULL) receives the index of
 * the first new variable; the others follow consecutively. */
int32_t pccp_model_add_vars(pccp_model *m, int32_t n, const int32_t *lb, const int32_t *ub,
                            int32_t *first_id);

/* Append the constraint sum_{t<nterms} coef[t] * x_{var[t]} <= rhs.
 * §2 compiles x + y <= c to the tells ub(x) <= c - lb(y), ub(y) <= c - lb(x)
 * and the resource sum to the tells on each b from the other terms; this
 * generalises both: with m_t the smallest value of a_t x_t over the store
 * and S = sum_t m_t, each x_t is told a_t x_t <= rhs - (S - m_t), rounded
 * toward the interval's inside.  Terms must be nonzero and name distinct
 * variables; nterms >= 1. */
int32_t pccp_model_add_linear_le(pccp_model *m, int32_t nterms, const int32_t *coef,
                                 const int32_t *var, int32_t rhs);

/* Append b <=> (si <= sj and sj < si + d), compiled as the four guarded
 * processes of §2 ([[phi <=> psi]]) with interval entailment; the negation
 * sj < si or sj >= si + d is propagated when one disjunct is entailed false.
 * b is read as true when lb(b) >= 1 and false when ub(b) <= 0. */
int32_t pccp_model_add_reified_overlap(pccp_model *m, int32_t b, int32_t si, int32_t sj,
                                       int32_t d);

/* Append the guarded command {g_1, ..., g_n} => x <- f of the guarded
 * normal form (§3: a program is a set of commands whose guards are
 * entailment tests and whose bodies are tells; §2: ask and tell), with
 *   f = k + sum_{t < nterms} coef[t] * y_{var[t]},
 *   side 0: lb(x) >= ceil(f / div),  side 1: ub(x) <= floor(f / div),
 * div >= 1.  Guard g tests one bound: gside[g] = 0 is entailed(y >= gc[g])
 * = lb(y) >= gc[g], gside[g] = 1 is entailed(y <= gc[g]) = ub(y) <= gc[g]
 * (y = gvar[g]).  The tell runs when every guard holds (nguards = 0: always)
 * and each term is read through the bound that keeps f monotone as the
 * store grows (§2: tells are monotone): for a lower-bound tell lb(y) when
 * coef > 0 and ub(y) when coef < 0, the opposite for an upper-bound tell.
 * Read on points, the command says: if every guard holds then div * x >= f
 * (side 0) or div * x <= f (side 1).  Checked when a solver is created:
 * indices in range, side in {0, 1}, div >= 1, nonzero coefficients,
 * |k| + sum |coef| * max |bound| < 2^30 (PCCP_E_OVERFLOW), at most 65535
 * guards and 65535 terms per command. */
int32_t pccp_model_add_guarded(pccp_model *m, int32_t x, int32_t side, int32_t k, int32_t div,
                               int32_t nguards, const int32_t *gvar, const int32_t *gside,
                               const int32_t *gc, int32_t nterms, const int32_t *coef,
                               const int32_t *var);

/* Branching candidates, in tie-break order (§1: the search splits on them). */
int32_t pccp_model_set_decision_vars(pccp_model *m, int32_t n, const int32_t *vars);

/* Variable to minimise (-1 = none).  A solution's value is lb(objective). */
int32_t pccp_model_set_objective(pccp_model *m, int32_t var);

/* Sizes of a model: any pointer may be NULL. */
int32_t pccp_model_info(const pccp_model *m, int32_t *nvars, int32_t *nlinear,
                        int32_t *nterms, int32_t *nreified, int32_t *ndecision);

/* Model files: the variables, constraints, decision list and objective of a
 * model (§2 modelling layer, after compilation to the two constraint forms;
 * §3 names erased to indices), so that a generated model is built once and
 * read by every consumer.  Layout, all integers little-endian:
 *   line 1   "PCCP-MODEL 1"
 *   line 2   a JSON object with the integer fields nvars, nrows, nterms,
 *            nreif, ndec, objective, and optionally ncmd, nguards, ncterms
 *            (absent = 0); other fields are ignored on load (a generator
 *            may add its parameters there)
 *   then     int32 lb[nvars], ub[nvars], row_ptr[nrows + 1] (0 .. nterms,
 *            increasing), coef[nterms], var[nterms], rhs[nrows],
 *            reif[4 * nreif] (b, si, sj, d per item), dec[ndec]
 *   and, when ncmd > 0, the guarded commands: cmd[4 * ncmd] (x, side, k,
 *            div), cmd_gptr[ncmd + 1] (0 .. nguards, not decreasing),
 *            guard[3 * nguards] (y, side, c), cmd_tptr[ncmd + 1] (0 ..
 *            ncterms, not decreasing), cterm[2 * ncterms] (coef, y)
 * save writes the model as built; load creates a model (*out, destroyed with
 * pccp_model_destroy) or returns PCCP_E_MODEL for a bad header, a file of
 * the wrong length or an inconsistent row pointer, PCCP_E_INVALID_ARG if the
 * file cannot be opened.  Index ranges are checked when a solver is
 * created, as for a model built call by call. */
int32_t pccp_model_save_file(const pccp_model *m, const char *path);
int32_t pccp_model_load_file(const char *path, pccp_model **out);

/* ---- solver ------------------------------------------------------------ */
/* A zero-initialised pccp_config selects every default. */
typedef struct {
    int32_t wg_size;      /* threads per workgroup, multiple of 64, <= 1024;
                             0 = 256                                          */
    int32_t num_wgs;      /* workgroups of a search launch; 0 = as many as are
                             resident at once on the device                   */
    int32_t desc_lds;     /* propagator tables: 0 = choose, 1 = copy into
                             LDS, 2 = read from global memory                 */
    int32_t root_lds;     /* subtree-root store: 0 = choose, 1 = LDS,
                             2 = global memory                                */
    int32_t max_depth;    /* decision-stack capacity per workgroup; 0 = 1024
                             (levels live in device memory, the deepest 256
                             also in LDS: capacity costs no LDS)          */
    int32_t queue_cap;    /* subtree queue slots; 0 = 4 x workgroups          */
    int64_t sol_cap;      /* ENUMERATE: solutions kept (all are counted)      */
    int32_t launch;       /* 0 = one hipGraph (initialisation + search
                             kernels, re-used while the launch parameters are
                             unchanged), 1 = two plain kernel launches        */
    int32_t live;         /* item lists: 1 = on; 0 (default) or 2 = off.  On: a
                             propagator found entailed at a node (no tell of
                             it can tighten that store or any tighter one) is
                             left out of the sweeps below that node; fixed
                             points, and so the search tree, are unchanged
                             (Theorem 2 of section 3); the lists take three
                             LDS buffers of 2 bytes per propagator          */
    int32_t occupancy;    /* search kernel build: 0 = choose (high for
                             wg_size <= 256), 1 = high (at least 7 waves per
                             SIMD, 6 with dep = 1; wg_size <= 256, leaner
                             unrolling),
                             2 = normal (any wg_size)                       */
    int32_t dep;          /* dependency-driven propagation: 1 = on; 0
                             (default) or 2 = off.  On: after the first sweep
                             of a node, a sweep runs only the propagators that
                             read a bound tightened in the sweep before (the
                             improvement of the naive loop that section 6
                             points to; the fixed point is unchanged,
                             Theorem 2 of section 3), and a backtrack
                             restores the parent's store from a trail in
                             global memory instead of recomputing it from
                             the subtree root; excludes live = 1           */
    int32_t trail_cap;    /* trail entries per workgroup with dep = 1; 0 = 8
                             per store variable within [4096, 2^18].  A path
                             whose changes do not fit is recomputed from the
                             subtree root instead                          */
} pccp_config;

/* Validate the model, compile it to packed per-kind propagator tables and
 * upload them to the current device.  cfg may be NULL (defaults).  stream
 * is a hipStream_t (may be 0). */
int32_t pccp_solver_create(const pccp_model *m, const pccp_config *cfg, void *stream,
                           pccp_solver **out);
int32_t pccp_solver_destroy(pccp_solver *s);

/* Fixed point (§3, Theorem 2) of the box (lb_in, ub_in) - host arrays of
 * nvars values, or both NULL for the model's initial box - computed by one
 * workgroup with every propagator running concurrently (§5, fixed point
 * loop).  *status receives PCCP_FIXPOINT or PCCP_FAILED.  The store is kept
 * for pccp_get_domains.  Synchronises the solver's stream. */
int32_t pccp_propagate(pccp_solver *s, const int32_t *lb_in, const int32_t *ub_in,
                       int32_t *status);

/* Copy the store of the last pccp_propagate (cap >= nvars). */
int32_t pccp_get_domains(pccp_solver *s, int32_t *lb, int32_t *ub, int32_t cap);

/* Fixed points of nbox boxes at once, one workgroup per box.  All pointers
 * are device memory: lb_in/ub_in/lb_out/ub_out are [nbox][nvars] int32
 * (row-major), status is [nbox] (PCCP_FIXPOINT / PCCP_FAILED), sweeps is
 * [nbox] (loop iterations, may be NULL).  On a failed box lb_out/ub_out are
 * unspecified.  Enqueued on the solver's stream; returns without waiting. */
int32_t pccp_propagate_batch(pccp_solver *s, int32_t nbox, const int32_t *lb_in,
                             const int32_t *ub_in, int32_t *lb_out, int32_t *ub_out,
                             int32_t *status, int32_t *sweeps);

/* Incremental fixed points by dependency-driven propagation (§3, Theorem 2:
 * any fair schedule - here, running a propagator only after a bound it
 * reads was tightened - reaches the same least fixed point).  Box k is the
 * store (lb_in, ub_in) row k joined with one decision,
 *   lb(dvar[k]) >= dlo[k]  and  ub(dvar[k]) <= dhi[k]
 * (a join: a bound already tighter is kept).  Precondition: every input
 * store is a fixed point of the model, e.g. an output of
 * pccp_propagate_batch; then lb_out/ub_out row k is the fixed point of
 * the joined box, the one pccp_propagate_batch computes from it.  Only the
 * propagators that read a bound the decision tightened run in the first
 * sweep, and each later sweep runs those reading a bound the one before
 * tightened.  All pointers are device memory: lb_in/ub_in/lb_out/ub_out are
 * [nbox][nvars] int32, dvar/dlo/dhi/status/sweeps [nbox] (sweeps may be
 * NULL).  status[k] = PCCP_FIXPOINT, PCCP_FAILED (lb_out/ub_out row k
 * unspecified), or -1 when dvar[k] is outside [0, nvars) (the row is copied
 * unchanged).  PCCP_E_UNSUPPORTED if a kind has more than 65536
 * propagators.  Enqueued on the solver's stream; returns without
 * waiting. */
int32_t pccp_propagate_batch_incr(pccp_solver *s, int32_t nbox, const int32_t *lb_in,
                                  const int32_t *ub_in, const int32_t *dvar, const int32_t *dlo,
                                  const int32_t *dhi, int32_t *lb_out, int32_t *ub_out,
                                  int32_t *status, int32_t *sweeps);

/* Branching features (6 floats per decision variable, in decision-list
 * order) of nbox stores; all pointers are device memory: lb/ub are
 * [nbox][nvars] int32, feat is [nbox][ndecision][6] float.  For decision
 * variable x with initial interval [lo, hi], H = max(1, hi - lo):
 *   f0 = (lb(x) - lo)/H, f1 = (ub(x) - lo)/H, f2 = (ub(x) - lb(x))/H,
 *   f3 = (rows + reified items containing x) / the largest such count,
 *   f4 = min(1, min over rows x - y <= c of (c + ub(y) - lb(x))/H),
 *   f5 = mean over reified items with si = x of d * w(b) / H (w(b) = sum of
 *        a/c over rows a*b + ... <= c with a, c > 0) plus the fraction of
 *        those items with lb(b) >= 1.
 * These are the inputs of the learned branching rule (the paper leaves the
 * search strategy open, §5 Evaluation).  Decision variables must be
 * distinct.  Enqueued on the solver's stream. */
int32_t pccp_node_features(pccp_solver *s, int32_t nbox, const int32_t *lb, const int32_t *ub,
                           float *feat);

typedef struct {
    int64_t node_limit;           /* 0 = none; all instances of the launch     */
    double time_limit_s;          /* 0 = none; measured on the device clock    */
    const volatile int32_t *cancel; /* host word in pinned memory polled by the
                                     search (nonzero = stop); may be NULL     */
    int64_t inst_node_limit;      /* 0 = none; an instance that has used this
                                     many nodes is abandoned (outcome LIMIT)
                                     while the others go on, so a batch gives
                                     each instance the budget a plain search
                                     with node_limit would have; counted in
                                     steps of up to 256 nodes per workgroup   */
} pccp_limits;

/* Propagate-and-search on this solver's model (§1, §5): mode is
 * PCCP_ENUMERATE or PCCP_MINIMIZE.  limits may be NULL.  One persistent
 * launch: every workgroup takes subtrees from a device queue and explores
 * them depth first; the subtree closest to a workgroup's root is donated to
 * the queue while others are idle.  With cfg.num_wgs = 1 the node order is
 * the sequential depth-first order.  *outcome receives a PCCP_OUT_* value.
 * Synchronises the solver's stream.  Returns PCCP_E_DEPTH if a path was
 * deeper than max_depth. */
int32_t pccp_solve(pccp_solver *s, int32_t mode, const pccp_limits *limits, int32_t *outcome);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * search as pccp_solve, on the same kernels, with the whole search
 * workspace (queue, per-instance state, decision stacks, trail, subtree
 * roots) taken from a static device array of 64 MiB that the library holds
 * on every device it is loaded on until the process ends.  It calls no
 * hipMalloc, hipFree or allocating library routine and launches the kernels
 * directly (no graph).  The solver (created beforehand) is the input; the
 * outcome, stats, best objective and values, solution count and hash are
 * the outputs, read with the usual calls.  The list of solutions is not
 * kept (pccp_get_solutions refuses any non-empty range).
 * Returns PCCP_E_NOMEM, before any device work, when the launch shape needs
 * more than 64 MiB (16 bytes x max_depth per workgroup for the stacks, plus
 * 16 bytes x trail_cap per workgroup with dependency-driven propagation, plus
 * the queue): lower cfg.num_wgs, max_depth or trail_cap.  Every call on a
 * device shares that device's array: calls that overlap on one GPU (two host
 * threads, two streams) race and give wrong results.  The array keeps the
 * last call's contents; each call initialises what it reads. */
int32_t pccp_solve_noalloc(pccp_solver *s, int32_t mode, const pccp_limits *limits,
                           int32_t *outcome);

/* The same search over n solvers' models in ONE persistent launch (one
 * shared queue; instances of different sizes).  All solvers must live on
 * the current device; the launch uses solvers[0]'s stream and cfg (may be
 * NULL = solvers[0]'s).  outcomes[i] receives solver i's outcome, and each
 * solver's stats/best/solutions are updated as if it had been solved
 * alone. */
int32_t pccp_batch_solve(pccp_solver *const *solvers, int32_t n, int32_t mode,
                         const pccp_config *cfg, const pccp_limits *limits, int32_t *outcomes);

typedef struct {
    int64_t nodes;            /* propagate calls of the search (failed ones and
                                 solutions included)                          */
    int64_t fails;
    int64_t solutions;        /* ENUMERATE: solutions; MINIMIZE: improvements */
    int64_t sweeps;           /* propagation-loop iterations, all nodes       */
    int64_t donations;        /* subtrees given to the queue                  */
    int64_t subtrees;         /* subtrees taken from the queue                */
    int64_t max_depth;
    int64_t prop_linear2;     /* propagator executions: difference rows       */
    int64_t prop_reified;     /*                         reified overlaps     */
    int64_t prop_linear;      /*                         other linear rows and
                                                         guarded commands     */
    int64_t prop_terms;       /* terms visited by other linear rows           */
    uint64_t sol_hash;        /* ENUMERATE: wrapping sum over solutions of
                                 fmix64(FNV-1a-64(decision values, LE bytes)) */
    int32_t best;             /* MINIMIZE: best objective (INT32_MAX = none)  */
    int32_t outcome;          /* PCCP_OUT_*                                   */
    double kernel_ms;         /* duration of the search kernel (HIP events)   */
    double ttpo_ms;           /* device clock, search start -> last subtree
                                 finished; -1 if not finished                 */
    int32_t grid, block, desc_lds, root_lds;
    int64_t lds_bytes;
    int32_t live;             /* the search kept item lists                   */
    int32_t occupancy;        /* 1 = high-occupancy build, 2 = normal         */
    int32_t dep;              /* dependency-driven propagation with a trail   */
    int32_t pad;
    int64_t atomics;          /* lattice joins issued by the sweeps: one LDS
                                 atomic max (lb) or min (ub) per tell whose
                                 value was strictly tighter than the bound the
                                 lane read (§4: store only on a strict gain;
                                 §5 erratum: the store's joins are atomic)    */
} pccp_stats;

int32_t pccp_get_stats(const pccp_solver *s, pccp_stats *st);

/* ENUMERATE: number of solutions found (counted even beyond sol_cap). */
int32_t pccp_get_solution_count(const pccp_solver *s, int64_t *count);

/* ENUMERATE: order-independent hash of the solution set found by the last
 * search: the wrapping sum over solutions of fmix64 (MurmurHash3's final
 * mix) of the 64-bit FNV-1a hash of the decision values' little-endian
 * bytes, so that searches splitting the tree differently can be compared
 * (§5: subproblems explored in any order).  PCCP_E_STATE before a search. */
int32_t pccp_get_solution_hash(const pccp_solver *s, uint64_t *hash);

/* ENUMERATE: copy solutions [first, first + count) (ndecision values each,
 * in the order they were found) into vals.  Only the first sol_cap are
 * kept. */
int32_t pccp_get_solutions(pccp_solver *s, int64_t first, int64_t count, int32_t *vals);

/* MINIMIZE: best objective (*obj = INT32_MAX if none) and the decision
 * values of that solution (cap >= ndecision). */
int32_t pccp_get_best(pccp_solver *s, int32_t *obj, int32_t *vals, int32_t cap);

/* Branching rule for later searches: PCCP_BRANCH_*.  For PCCP_BRANCH_MLP,
 * weights is the device pointer given by pccp_mlp_weights (the network must
 * outlive the searches that use it); NULL falls back to first-fail. */
int32_t pccp_set_branching(pccp_solver *s, int32_t kind, const void *weights);

/* Number of workgroups of each configuration that are resident at once
 * (the default grid of a search launch). */
int32_t pccp_solver_capacity(const pccp_solver *s, int32_t *wgs_per_cu, int32_t *num_cus);

/* ---- launch tuning ------------------------------------------------------
 * The paper picks its launch shape by measurement (§5 Evaluation: 4x
 * oversubscription of the GPU's blocks was best on its machine).  The tuner
 * times short searches of the given models in one launch under each
 * candidate configuration - workgroup size x propagator tables in LDS or
 * global memory x subtree-root store in LDS or global memory x propagation
 * mode x kernel build - and returns the fastest (nodes per second of device
 * time).  A zero-initialised pccp_tune_opts selects every default. */
typedef struct {
    double budget_s;      /* device-clock seconds of one probe; 0 = 0.4      */
    int32_t whole_run;    /* 0: steady-state rate - the nodes and device time
                             of a run of budget_s / 2 are subtracted from
                             those of a run of budget_s, so the start-up
                             while the queue fills cancels out (unless the
                             searches finish early); 1: the whole run's rate
                             (what searches to a quick proof see)           */
    int32_t finalists;    /* the best this many are timed again with runs 4x
                             as long; rates within 2 % count as ties, won by
                             the better first-pass rank; 0 = 3              */
    int32_t modes;        /* propagation modes tried, bit mask: 1 every table
                             every sweep, 2 dependency-driven, 4 item lists;
                             0 = 1 | 2                                      */
    int32_t wg_sizes;     /* workgroup sizes tried, bit k = 64 << k (k = 0..4);
                             0 = 128, 256, 512 and 1024                     */
    int32_t max_depth;    /* decision-stack capacity of every candidate;
                             0 = solvers[0]'s                               */
    int32_t pad;
} pccp_tune_opts;

typedef struct {
    pccp_config cfg;          /* the candidate                              */
    double nodes_per_s;       /* first-pass rate (0 when status != PCCP_OK)  */
    double nodes_per_s_long;  /* rate of the long runs (finalists), else 0   */
    int32_t grid;             /* workgroups the candidate's launch used      */
    int32_t status;           /* PCCP_OK, PCCP_E_LDS_CAPACITY (the layout
                                 does not fit) or PCCP_E_DEPTH (a path was
                                 deeper than max_depth)                      */
} pccp_tune_result;

/* Tune the launch for searching solvers[0..n) together in `mode` (every
 * probe is a pccp_batch_solve with a time limit, so their stats are those
 * of the last probe).  *best receives the chosen configuration (its
 * num_wgs, queue_cap, sol_cap, launch and trail_cap are solvers[0]'s).
 * results (may be NULL) receives up to cap candidates in the order tried,
 * *nresults (may be NULL) their number.  Returns PCCP_E_LDS_CAPACITY if no
 * candidate fits, or the first other error a probe gave. */
int32_t pccp_autotune(pccp_solver *const *solvers, int32_t n, int32_t mode,
                      const pccp_tune_opts *opts, pccp_config *best,
                      pccp_tune_result *results, int32_t cap, int32_t *nresults);

/* ---- floating-point interval stores -----------------------------------
 * §2 defines the lattices FInc and FDec of increasing and decreasing
 * floating-point numbers, ordered by the IEEE 754 total order (footnote);
 * §6 notes that intervals of reals are approximated by intervals of floats.
 * A float model has float32 interval variables (lb in FInc, ub in FDec) and
 * linear rows over the reals, sum_t coef[t] * x_var[t] <= rhs.  Each term's
 * tell is the linear tell of §2 with outward rounding, so that no real
 * solution is removed: the other terms' least values a_u * (lb or ub)(x_u)
 * rounded down and summed in term order from +0 with each addition rounded
 * down (S), then ub(x_t) <- (rhs - S, rounded up) / a_t rounded up when
 * a_t > 0, lb(x_t) <- (rhs - S, rounded up) / a_t rounded down when a_t < 0.
 * Zero bounds are canonical: a lower bound of zero is -0 and an upper bound
 * of zero is +0 (so the total order and the numeric one agree).  A box is
 * failed when some lb > ub. */

/* Empty float model / destroy. */
int32_t pccp_fmodel_create(pccp_fmodel **out);
int32_t pccp_fmodel_destroy(pccp_fmodel *m);

/* Append n variables with initial intervals [lb[i], ub[i]] (finite;
 * checked at pccp_fsolver_create).  *first_id (may be NULL) receives the
 * index of the first. */
int32_t pccp_fmodel_add_vars(pccp_fmodel *m, int32_t n, const float *lb, const float *ub,
                             int32_t *first_id);

/* Append sum_{t<nterms} coef[t] * x_{var[t]} <= rhs (nterms >= 1; nonzero
 * finite coefficients, distinct variables, finite rhs; checked at
 * pccp_fsolver_create). */
int32_t pccp_fmodel_add_linear_le(pccp_fmodel *m, int32_t nterms, const float *coef,
                                  const int32_t *var, float rhs);

/* Validate the float model and upload its tables to the current device
 * (the rows in order of their length, and slot-major copies of the terms of
 * rows of up to 8 terms: 8 bytes per term plus 140 bytes per row).
 * wg_size: threads per workgroup (multiple of 64, <= 1024; 0 = 256).
 * PCCP_E_MODEL for a non-finite bound or coefficient, a zero coefficient,
 * an index out of range or a variable repeated in a row;
 * PCCP_E_LDS_CAPACITY if 8 bytes per variable do not fit in LDS. */
int32_t pccp_fsolver_create(const pccp_fmodel *m, int32_t wg_size, void *stream,
                            pccp_fsolver **out);
int32_t pccp_fsolver_destroy(pccp_fsolver *s);

/* Fixed points of nbox float boxes, one workgroup per box, one lane per
 * row running its terms' tells concurrently with the other rows' (LDS
 * atomic max / min on the bounds' total-order keys; §5 fixed point loop on
 * the float lattices).  The tells are
 * monotone, so the result is the least fixed point (§3, Theorem 2): the
 * same store, bit for bit, as a sequential loop.  All pointers are device
 * memory: lb_in/ub_in/lb_out/ub_out are [nbox][nvars] float32 (zeros of the
 * inputs are made canonical), status [nbox] receives PCCP_FIXPOINT or
 * PCCP_FAILED (on FAILED the output row is unspecified), sweeps [nbox] (may
 * be NULL) the loop's iterations.  Enqueued on the solver's stream. */
int32_t pccp_fpropagate_batch(pccp_fsolver *s, int32_t nbox, const float *lb_in,
                              const float *ub_in, float *lb_out, float *ub_out,
                              int32_t *status, int32_t *sweeps);

/* ---- LDS peaks ----------------------------------------------------------
 * The propagation loop's store lives in LDS (§5: the shared-memory store was
 * the fastest; its joins are atomic per the erratum), so its roofline is
 * LDS bandwidth and LDS atomic throughput.  This measures both on the
 * current device with conflict-free access patterns over every compute
 * unit: 64-bit LDS reads (ds_read_b64), and 32-bit atomic max without and
 * with the old value returned.  Synchronises the null stream. */
typedef struct {
    double read_gbs;          /* LDS bytes read per second / 1e9             */
    double atomic_gops;       /* LDS atomic max lane operations per second,
                                 no return, / 1e9                            */
    double atomic_ret_gops;   /* the same with the old value returned        */
    double ms[3];             /* kernel times of the three measurements      */
    int32_t num_cus;
    int32_t grid, block;      /* launch of each measurement                  */
    int32_t pad;
} pccp_lds_peaks;

int32_t pccp_measure_lds_peaks(pccp_lds_peaks *out);

/* ---- learned branching: network and training --------------------------
 * The rule scores each unfixed decision variable from its 6 features
 * (pccp_node_features) with a 2-layer network: s = w2 . max(0, W1 x + b1)
 * + b2, 64 hidden units; the search branches on the largest score (ties to
 * the earliest decision variable).  Parameters (513 floats): W1[k][f] at
 * k*6+f, b1 at 384+k, w2 at 448+k, b2 at 512.  Training keeps FP32 master
 * weights and Adam moments on the device; the search reads a BF16 copy and
 * accumulates in FP32.  Targets come from search traces (how strongly an
 * expert prefers each candidate of a node); the loss is the mean over nodes
 * of the cross-entropy between target and softmax over the candidates.  The paper leaves the
 * search strategy open (§5, Evaluation); first-fail is the fallback. */
typedef struct pccp_mlp pccp_mlp;

/* New network on the current device, Glorot-uniform weights drawn from a
 * SplitMix64 stream seeded with `seed`, zero biases.  stream: hipStream_t. */
int32_t pccp_mlp_create(uint64_t seed, void *stream, pccp_mlp **out);
int32_t pccp_mlp_destroy(pccp_mlp *m);

/* Host copies of the 513 FP32 parameters; set also resets the Adam state. */
int32_t pccp_mlp_set_params(pccp_mlp *m, const float *params);
int32_t pccp_mlp_get_params(pccp_mlp *m, float *params);

/* One training step on device data: feat [ncand][6] float, node_off
 * [nnodes+1] int32 (candidates of node i are node_off[i]..node_off[i+1]-1),
 * target [ncand] float (a distribution over each node's candidates: the
 * loss is the mean over nodes of -sum_c target_c log softmax(s)_c),
 * max_cand = the largest candidate count of a node (<= 256).  Computes the
 * loss and gradient at the current parameters, then (lr > 0) one Adam step
 * (beta 0.9/0.999, eps 1e-8) and refreshes the BF16 copy.  *loss (may be
 * NULL) receives the loss before the step (synchronises the stream). */
int32_t pccp_mlp_train_step(pccp_mlp *m, const float *feat, const int32_t *node_off,
                            const float *target, int32_t nnodes, int32_t ncand,
                            int32_t max_cand, float lr, float *loss);

/* Gradient (513 floats, host) of the last training step. */
int32_t pccp_mlp_get_grads(pccp_mlp *m, float *grads);

/* Scores of ncand candidates (device arrays feat [ncand][6], scores
 * [ncand]) with the FP32 master weights (bf16 = 0) or the BF16 copy the
 * search uses (bf16 = 1). */
int32_t pccp_mlp_scores(pccp_mlp *m, const float *feat, int32_t ncand, float *scores,
                        int32_t bf16);

/* Device pointer of the BF16 parameters, for pccp_set_branching. */
int32_t pccp_mlp_weights(const pccp_mlp *m, const void **weights);

const char *pccp_last_error(void);
const char *pccp_version(void);

#ifdef __cplusplus
}
#endif
#endif
