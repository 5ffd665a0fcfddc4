// Device-side data layout shared by the C-ABI host code and the HIP kernels
// of libpccp.  Not part of the public interface (include/pccp.h is).
//
// One instance = one flattened model (§2: constraints compiled to
// propagators, names erased to store indices as in §3) uploaded once.  Each
// propagator kind is a structure-of-arrays table of packed descriptors so
// that a wavefront reads 64 consecutive descriptors with coalesced loads.
// Variable indices fit in 16 bits because a store must fit in one
// workgroup's LDS (8 bytes per variable, 160 KiB per CU).
#pragma once
#include <stdint.h>

namespace pccp {

constexpr int kMaxVars = 65535;
constexpr int kMaxWg = 1024;
constexpr int kCtlWords = 96;   // LDS control block (int32 words)

// Kind 1 - difference row  x - y <= c  (a linear row with coefficients
// +1 / -1; every precedence s_i + d_i <= s_j is one).
//   packed.x = x | (y << 16),  packed.y = c
// Kind 2 - reified overlap  b <=> (si <= sj  and  sj < si + d).
//   packed.x = b | (si << 16), packed.y = sj | (d << 16)   (d as int16)
// Kind 3 - general linear row  sum_t a_t x_t <= rhs.
//   row = {first term, number of terms, rhs, 0}; term = var | (a << 16)
//   (a as int16, nonzero)
// Kind 4 - Boolean knapsack row  sum_t a_t b_t <= rhs, every b_t with an
//   initial domain inside [0, 1] and every a_t > 0 (kind 3's rule on 0/1
//   domains).  row = {rhs, number of terms}; terms row-major with a fixed
//   stride of bgroup * bchunks slots per row, term = var | (a << 16), the
//   unused slots of a row hold 0 (a = 0).
// Kind 5 - guarded command  {g_1, ..., g_n} => x <- f  (§3, guarded normal
//   form), f = k + sum_t a_t y_t: when every guard is entailed (guard
//   (y, 0, c): lb(y) >= c; (y, 1, c): ub(y) <= c), side 0 joins
//   ceil(f / div) into lb(x), side 1 joins floor(f / div) into ub(x), each
//   term read through the bound that keeps f monotone.
//   cmd = {x | side << 16, k, div, first entry}; cnt = guards | terms << 16;
//   entries: the guards {y | side << 16, c}, then the terms
//   {y | (reads ub) << 16, a}.
// The store of one instance (see Store in the kernels): the variables whose
// initial domain is not inside [0, 1] first, as (lb, ub) int32 pairs
// (indices [0, nI)), then the Booleans, one byte each (indices [nI, nvars)).
// The compiled model numbers its variables in that order; vorig / vnew map
// between that numbering and the model's own.
__host__ __device__ inline int store_pairs(int nI) { return (nI + 1) & ~1; }
__host__ __device__ inline int store_bool_words(int nI, int nvars)
{
    return (((nvars - nI) + 3) / 4 + 3) & ~3;
}
__host__ __device__ inline size_t store_bytes(int nI, int nvars)
{
    return 8 * (size_t)store_pairs(nI) + 4 * (size_t)store_bool_words(nI, nvars);
}

struct DevModel {
    int32_t nvars;
    int32_t nI;                   // variables stored as int32 pairs (the others are Booleans)
    int32_t ndiff, nreif, nrows, nterms;
    int32_t ndec, objective;
    int32_t row_group;            // lanes per linear row in a sweep (4, 8 or 16)
    int32_t row_chunks;           // ceil(longest row / row_group)
    int32_t nbrows;               // kind 4 rows
    int32_t bgroup, bchunks;      // kind 4: lanes per row, term slots per lane
    int32_t nbterms;              // kind 4 terms (without the padding)
    int32_t ncmd;                 // kind 5 commands
    const int32_t *lb0, *ub0;     // initial box
    const int2 *diff;             // kind 1
    const int2 *reif;             // kind 2
    const int4 *rows;             // kind 3 rows
    const uint32_t *terms;        // kind 3 terms
    const int2 *brows;            // kind 4 rows {rhs, len}
    const uint32_t *bterms;       // kind 4 terms [nbrows * bgroup * bchunks]
    const int32_t *dec;           // decision variables (tie-break order)
    const int32_t *vorig;         // store index -> the model's variable index
    const int32_t *vnew;          // the model's variable index -> store index
    const int4 *cmds;             // kind 5 commands
    const uint32_t *ccnt;         // kind 5 guard and term counts
    const int2 *cent;             // kind 5 guards and terms
    // learned branching: per decision variable q, fstat[8q..8q+4] =
    // {lo, 1/H, degree share, static load, 1/N}; rows x - y <= c leaving
    // x = dec[q] as fr[fr_ptr[q]..fr_ptr[q+1]) = {y, c}; b of the reified
    // items with si = x as fb[fb_ptr[q]..fb_ptr[q+1])
    const float *fstat;
    const int32_t *fr_ptr;
    const int2 *fr;
    const int32_t *fb_ptr;
    const int32_t *fb;
    // dependency-driven propagation: the propagators that read variable x
    // are adj[adj_ptr[x]..adj_ptr[x+1]), entry = index in its kind's table
    // | kind << 16 (0 difference rows, 1 reified items, 2 linear rows,
    // 3 Boolean rows, 4 guarded commands) | reads lb(x) << 19 | reads ub(x) << 20
    const int32_t *adj_ptr;
    const uint32_t *adj;
};
constexpr uint32_t kAdjLb = 1u << 19;
constexpr uint32_t kAdjUb = 1u << 20;
constexpr int kDepKinds = 5;     // propagator kinds of the dependency-driven work lists

constexpr int kNumFeat = 6;
constexpr int kHidden = 64;
constexpr int kNumParams = kHidden * kNumFeat + kHidden + kHidden + 1;  // 513

// Per-instance search results, written by the search kernel.
struct InstState {
    unsigned long long nodes, fails, solutions, sweeps;
    unsigned long long donations, pops, sol_hash, max_depth;
    unsigned long long ex[4];   // propagator executions: difference rows,
                                // reified items, linear rows (kinds 3 and 4);
                                // row terms
    unsigned long long atomics; // lattice joins issued (LDS atomic max / min)
    long long t_done;           // wall-clock tick when the last subtree finished (0 = not done)
    int32_t best;               // MINIMIZE: best objective so far (INT32_MAX = none)
    int32_t outstanding;        // subtrees queued or in progress
    int32_t best_lock;          // spin lock protecting best_vals
    int32_t best_owner;         // workgroup that wrote best_vals
    int32_t depth_overflow;     // a path exceeded the decision-stack capacity
    int32_t pad[2];             // pad[0]: objective of best_vals (under best_lock)
    int32_t abandon;            // the instance used its node budget
};

// Queue slot header; a slot is followed by max_depth decisions (int2).
struct RecHdr {
    int32_t inst;
    int32_t len;
    int32_t pad[2];
};

// A decision on the search path.  word = var | (side << 16) | (donated << 17);
// side 0 = left child (ub(var) := val), side 1 = right child (lb(var) := val + 1).
constexpr uint32_t kSideBit = 1u << 16;
constexpr uint32_t kDonatedBit = 1u << 17;

struct SearchGlobals {
    unsigned long long q_head, q_tail;  // Vyukov bounded MPMC queue positions
    unsigned long long q_pushed;
    int32_t outstanding;                // all instances
    int32_t idle;                       // workgroups waiting for work
    int32_t abort;                      // 1 = node limit, 2 = time limit, 3 = cancelled, 4 = stack overflow
    int32_t pad;
    unsigned long long nodes_total;     // flushed periodically, for the node limit
    long long t_start;                  // wall_clock64() when the search was initialised
};

// Incremental fixed points: box k is the fixed point (lb_in, ub_in) joined
// with lb(dvar[k]) >= dlo[k] and ub(dvar[k]) <= dhi[k]; the LDS layout of the
// dependency-driven loop as in SearchParams (dep_*).
struct IncrParams {
    int32_t nbox;
    int32_t dep_vshift, dep_qw, dep_jcap;
    int32_t dep_wcap[kDepKinds];
    const int32_t *lb_in, *ub_in;
    const int32_t *dvar, *dlo, *dhi;
    int32_t *lb_out, *ub_out;
    int32_t *status, *sweeps;
};

struct SearchParams {
    const DevModel *models;     // [ninst]
    InstState *inst;            // [ninst]
    int32_t ninst;
    int32_t mode;               // 0 enumerate, 1 minimise
    int32_t branching;          // 0 first-fail, 1 input order, 2 MLP
    int32_t max_depth;          // decision stack capacity
    SearchGlobals *g;
    unsigned long long *q_seq;  // [qcap]
    char *q_data;               // [qcap * slot_bytes]
    int32_t qcap;
    int32_t slot_bytes;
    char *root_scratch;         // [grid * max_store] (global subproblem root stores)
    int32_t max_vars;           // largest instance in the launch (variables)
    int32_t pad1;
    long long max_store;        // bytes of the largest store (store_bytes) in the launch
    int32_t donate;             // allow donation (0 in single-workgroup runs)
    long long node_limit;       // 0 = none
    long long inst_node_limit;  // 0 = none: nodes per instance before it is abandoned
    long long t_limit_ticks;    // 0 = none (wall_clock64 ticks)
    const volatile int32_t *cancel;   // host-visible cancel word (may be null)
    int32_t *sol_buf;           // ENUMERATE: solutions (ndec values each)
    long long sol_cap;
    int32_t *best_vals;         // [ninst * max_ndec]
    int32_t max_ndec;
    int32_t pad;
    const uint16_t *mlp;        // learned branching: bf16 parameters (513), or null
    int32_t max_items[4];       // largest table per kind in the launch (item lists)
    // dependency-driven propagation (see the search kernel): variable
    // bitmaps of 1 << dep_vshift words (x at word x & mask, bit x >> shift),
    // dep_qw words of propagator marks, work lists of dep_wcap[k] entries,
    // and a trail of tcap entries per workgroup in global memory
    int32_t dep_vshift, dep_qw;
    int32_t dep_wcap[kDepKinds];
    int4 *trail;                // [grid * tcap] {x, lb, ub, 0}
    int32_t tcap;
    int32_t dep_jcap;           // job-list entries of the two-phase expansion (0: one phase)
    int4 *gstack;               // decision stacks, [grid * max_depth]
};

}  // namespace pccp
