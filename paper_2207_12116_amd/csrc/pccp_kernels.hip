// HIP kernels of libpccp for gfx950 (CDNA4): lock-free parallel propagation
// to a fixed point over int32 interval stores, and depth-first
// propagate-and-search over a device-side queue of subtrees.
//
// Design (the paper's own GPU solver, §5, was written for a Turing laptop
// GPU; this keeps what holds on gfx950 and changes the rest):
//   * One workgroup per subproblem (§5: one block per subproblem).  The
//     store of the subproblem lives in LDS: each integer variable as one
//     (lb, ub) int32 pair (one 64-bit LDS read fetches both bounds), each
//     Boolean (initial domain within [0, 1]) as one byte (bit 0: lb = 1,
//     bit 1: ub = 0), joined with an LDS atomic OR.
//   * Two propagation modes.  Every table every sweep (eventless, §5): each
//     lane takes descriptors t = tid, tid + W, ... of each kind in turn (§5,
//     fixed point loop: strided loop over the propagators).  Dependency-
//     driven (the improvement §6 names): a sweep runs only the propagators
//     that read a bound the previous sweep tightened, found through a
//     variable -> propagator adjacency, whose entries each wavefront lays
//     out for a batch of changed variables at once; the same least fixed
//     point by chaotic iteration (§3 Theorem 2).
//   * A tell is a lattice join: LDS atomic max on lb, atomic min on ub
//     (ds_max_i32 / ds_min_i32, no return).  The plain load + compare +
//     store of the load/store compilation (§4) can lose an update when two
//     lanes write the same bound; the atomic join cannot.  Reads are
//     relaxed atomic loads, which satisfies the atomicity assumption (ATOM)
//     of §4 and the erratum of §5.  A tell is only issued when its value is
//     strictly tighter than the bound the lane read (§4: store only if the
//     joined value is greater).
//   * Fixed-point detection: the change and failure bits of a sweep are
//     OR-ed per wavefront with a ballot and published by lane 0 into one of
//     three rotating LDS words; one barrier per sweep (§5, has_changed[3]),
//     and one more after the work-list expansion in the dependency-driven
//     mode.  The barrier is an LDS-only fence + s_barrier, so global loads
//     issued by the control lane stay in flight across sweeps.
//   * Failure (an empty interval, §5) is flagged in-loop whenever a tell
//     crosses the opposite bound it read, which bounds the number of sweeps
//     on failing stores, and confirmed by a scan of the store at the fixed
//     point (§5: failure can be examined after the loop).
//   * Search (§5): each workgroup keeps the fixed point of its
//     subproblem's root.  Descending keeps the current store.  A backtrack
//     either undoes the path's changes from a trail (dependency-driven mode:
//     the first tell of a node on a variable saves the bounds it had) or,
//     where the trail overflowed or in the other modes, recomputes: copies
//     the root back and re-applies the decisions of the new path (§5: full
//     recomputation).  Embarrassingly parallel search with dynamically
//     generated subproblems (§5): a workgroup donates the right branch
//     closest to its subproblem root to a bounded lock-free MPMC queue when
//     other workgroups are idle.
//
// No MFMA: the work is integer lattice arithmetic, bound by the latency of
// dependent LDS and L2 round trips and of barriers.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "pccp_launch.h"
#include "pccp_types.h"

namespace pccp {

// ------------------------------------------------------------------ helpers
__device__ __forceinline__ int32_t lds_ld(const int32_t *p)
{
    return __hip_atomic_load(const_cast<int32_t *>(p), __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void join_lb(int32_t *p, int32_t v)
{
    __hip_atomic_fetch_max(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void join_ub(int32_t *p, int32_t v)
{
    __hip_atomic_fetch_min(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// The store of a subproblem.  A variable whose initial domain is not inside
// [0, 1] is the pair p[x] = (lb, ub), so one 64-bit LDS read fetches both
// bounds, and each half is joined on its own by a 32-bit atomic max / min
// (the 64-bit read is single-copy atomic per half, which is all a
// propagator needs: it may see one bound newer than the other, as with two
// reads).  A Boolean (initial domain inside [0, 1]; store indices nI and
// up) is one byte of the words b: bit 0 set means lb = 1, bit 1 set means
// ub = 0, both set the empty interval.  Both of a Boolean's tells are then
// atomic ORs (the join of the two-bit lattice), and a Boolean costs one
// byte of LDS instead of eight: the reified overlaps of the scheduling
// models have n^2 Booleans against n + 1 integers, so the store of a
// 120-task instance shrinks from 113 KiB to 15 KiB.  Tells of values
// outside [0, 1] on a Boolean empty it, as they would an interval.
struct Store {
    int2 *p;          // pairs [0, nI)
    uint32_t *b;      // Boolean bytes: variable x >= nI at byte x - nI
    int nI;
};

__device__ __forceinline__ Store make_store(char *base, int nI)
{
    Store s;
    s.p = reinterpret_cast<int2 *>(base);
    s.b = reinterpret_cast<uint32_t *>(base + 8 * (size_t)store_pairs(nI));
    s.nI = nI;
    return s;
}

__device__ __forceinline__ int2 dom(const Store st, int x)
{
    if (x < st.nI) {
        const unsigned long long u =
            __hip_atomic_load(reinterpret_cast<unsigned long long *>(st.p + x),
                              __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        return make_int2((int32_t)(uint32_t)u, (int32_t)(uint32_t)(u >> 32));
    }
    const uint32_t y = (uint32_t)(x - st.nI);
    const uint32_t w = __hip_atomic_load(st.b + (y >> 2), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    const uint32_t c = w >> (8 * (y & 3u));
    return make_int2((int32_t)(c & 1u), (int32_t)((~c >> 1) & 1u));
}
// the bits of a Boolean for the interval (lb, ub) (only ever a non-empty
// one, or one emptied by a bound beyond [0, 1])
__device__ __forceinline__ uint32_t bool_bits(int32_t lb, int32_t ub)
{
    return (lb >= 1 ? 1u : 0u) | (ub <= 0 ? 2u : 0u) | (lb >= 2 || ub < 0 ? 3u : 0u);
}
__device__ __forceinline__ void bool_or(const Store st, int x, uint32_t bits)
{
    const uint32_t y = (uint32_t)(x - st.nI);
    __hip_atomic_fetch_or(st.b + (y >> 2), bits << (8 * (y & 3u)), __ATOMIC_RELAXED,
                          __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void tell_lb(const Store st, int x, int32_t v)
{
    if (x < st.nI) join_lb(reinterpret_cast<int32_t *>(st.p) + 2 * x, v);
    else if (v >= 1) bool_or(st, x, v >= 2 ? 3u : 1u);
}
__device__ __forceinline__ void tell_ub(const Store st, int x, int32_t v)
{
    if (x < st.nI) join_ub(reinterpret_cast<int32_t *>(st.p) + 2 * x + 1, v);
    else if (v <= 0) bool_or(st, x, v < 0 ? 3u : 2u);
}
// write a variable's interval (no concurrent tell on the same variable; a
// Boolean's byte is written alone, its neighbours are untouched)
__device__ __forceinline__ void set_dom(const Store st, int x, int2 d)
{
    if (x < st.nI) {
        st.p[x] = d;
    } else {
        const uint32_t y = (uint32_t)(x - st.nI);
        reinterpret_cast<uint8_t *>(st.b)[y] = (uint8_t)bool_bits(d.x, d.y);
    }
}

__device__ __forceinline__ int uni(int x) { return __builtin_amdgcn_readfirstlane(x); }

// Lanes of the wavefront where p holds (wave-uniform).  The sweeps count the
// lattice joins (LDS atomic max / min) they issue with it, in code every
// lane of the wavefront runs, so the count stays in a scalar register.
__device__ __forceinline__ uint32_t lanes(bool p) { return (uint32_t)__popcll(__ballot(p)); }

// Barrier that orders LDS only (the store, flags and stack are all in LDS).
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Barrier that also orders global memory within the workgroup.
__device__ __forceinline__ void full_barrier() { __syncthreads(); }

template <typename T>
__device__ __forceinline__ T g_load(const T *p)
{
    return __hip_atomic_load(const_cast<T *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ T g_load_acq(const T *p)
{
    return __hip_atomic_load(const_cast<T *>(p), __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void g_store_rel(T *p, T v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ T g_add(T *p, T v)
{
    return __hip_atomic_fetch_add(p, v, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ bool g_cas(T *p, T &expected, T desired)
{
    return __hip_atomic_compare_exchange_strong(p, &expected, desired, __ATOMIC_ACQ_REL,
                                                __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Explicit global-address-space loads/stores (a generic pointer would make
// the compiler emit flat instructions, which also wait on the LDS counter).
typedef int v2i __attribute__((ext_vector_type(2)));
typedef int v4i __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) const v2i g_v2i;
typedef __attribute__((address_space(1))) const v4i g_v4i;
typedef __attribute__((address_space(1))) const int32_t g_i32;
typedef __attribute__((address_space(1))) int32_t g_i32w;
__device__ __forceinline__ int2 gread(const int2 *p)
{
    const v2i v = *(g_v2i *)p;
    return make_int2(v.x, v.y);
}
__device__ __forceinline__ int4 gread(const int4 *p)
{
    const v4i v = *(g_v4i *)p;
    return make_int4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ int32_t gread(const int32_t *p) { return *(g_i32 *)p; }
typedef __attribute__((address_space(1))) const float g_f32;
__device__ __forceinline__ float gread_f(const float *p) { return *(g_f32 *)p; }
__device__ __forceinline__ uint32_t gread(const uint32_t *p) { return (uint32_t) * (g_i32 *)p; }
__device__ __forceinline__ void gwrite(int32_t *p, int32_t v) { *(g_i32w *)p = v; }
typedef __attribute__((address_space(1))) v4i g_v4iw;
__device__ __forceinline__ void gwrite4(int4 *p, int4 v)
{
    v4i w;
    w.x = v.x; w.y = v.y; w.z = v.z; w.w = v.w;
    *(g_v4iw *)p = w;
}

// floor(a / b) for b > 0 (C's '/' truncates toward zero)
__device__ __forceinline__ int32_t floor_div_pos(int32_t a, int32_t b)
{
    int32_t q = a / b;
    return (q * b != a && a < 0) ? q - 1 : q;
}

__device__ __forceinline__ unsigned long long wave_min_u64(unsigned long long v)
{
    for (int off = 32; off > 0; off >>= 1) {
        unsigned long long o = __shfl_xor(v, off, 64);
        v = o < v ? o : v;
    }
    return v;
}

// Control words in LDS (int32 index; the two 64-bit words are 8-aligned).
enum : int {
    C_FLAG0 = 0, C_FLAG1 = 1, C_FLAG2 = 2,  // rotating sweep flags
    C_POSTFAIL = 3,                         // failure found by the post scan
    C_KEY = 4,                              // 64-bit branching key (words 4, 5)
    C_SLOT = 6,                             // queue position taken (low) ...
    C_SLOT_HI = 7,                          // ... and high word, or -1 / -2
    C_STOP = 8,                             // abandon the current subproblem
    C_DEPTH = 9,                            // new depth after a backtrack (-1 = done)
    C_INST = 10, C_LEN = 11,
    C_SKIP = 27,                            // the record taken was dropped
    C_CNT = 12,                             // item-list counts: 5 words per list
                                            // (R, A, B) = 4 kinds, row terms
    C_DCNT = 12,                            // or work-list counts: 5 words per set
                                            // (2 sets), one per kind
    C_DTERMS = 22,                          // row terms the node's sweeps visited
                                            // (dependency-driven mode)
    C_TTOP = 26,                            // entries pushed on the trail (dependency-driven
    C_THI = 31,                             // deepest path level without a whole trail  only)
    C_JCNT = 28,                            // entries of the expansion's job list
    C_MAXW = 29,                            // deepest decision-stack level written (every mode)
    C_ATOM = 30,                            // lattice joins issued by the node's sweeps
};

// ------------------------------------------------------------ descriptors
// Descriptor tables of one instance, in LDS (DL) or in global memory.
template <bool DL>
struct View {
    int32_t nvars, ndiff, nreif, nrows, nterms, ndec, objective;
    int32_t row_group, row_chunks;
    int32_t nbrows, bgroup, bchunks, nbterms;
    int32_t ncmd;
    const int2 *diff_;
    const int2 *reif_;
    const int4 *rows_;
    const uint32_t *terms_;
    const int2 *brows_;
    const uint32_t *bterms_;
    const int32_t *dec_;
    const int32_t *adjp_;         // always global memory
    const uint32_t *adj_;
    const int4 *cmds_;            // guarded commands: always global memory
    const uint32_t *ccnt_;
    const int2 *cent_;
    // Indices are non-negative: taking them as unsigned lets a global load
    // use a uniform base plus a 32-bit per-lane offset.
    __device__ __forceinline__ int2 brows(int t) const { return DL ? brows_[(uint32_t)t] : gread(brows_ + (uint32_t)t); }
    __device__ __forceinline__ uint32_t bterms(int t) const { return DL ? bterms_[(uint32_t)t] : gread(bterms_ + (uint32_t)t); }
    __device__ __forceinline__ int2 diff(int t) const { return DL ? diff_[(uint32_t)t] : gread(diff_ + (uint32_t)t); }
    __device__ __forceinline__ int2 reif(int t) const { return DL ? reif_[(uint32_t)t] : gread(reif_ + (uint32_t)t); }
    __device__ __forceinline__ int4 rows(int t) const { return DL ? rows_[(uint32_t)t] : gread(rows_ + (uint32_t)t); }
    __device__ __forceinline__ uint32_t terms(int t) const { return DL ? terms_[(uint32_t)t] : gread(terms_ + (uint32_t)t); }
    __device__ __forceinline__ int32_t dec(int t) const { return DL ? dec_[(uint32_t)t] : gread(dec_ + (uint32_t)t); }
    __device__ __forceinline__ int32_t adjp(int x) const { return gread(adjp_ + (uint32_t)x); }
    __device__ __forceinline__ uint32_t adj(int t) const { return gread(adj_ + (uint32_t)t); }
    __device__ __forceinline__ int4 cmd(int t) const { return gread(cmds_ + (uint32_t)t); }
    __device__ __forceinline__ uint32_t ccnt(int t) const { return gread(ccnt_ + (uint32_t)t); }
    __device__ __forceinline__ int2 cent(int t) const { return gread(cent_ + (uint32_t)t); }
};

__host__ __device__ inline size_t align16(size_t x) { return (x + 15) & ~size_t(15); }

__host__ __device__ inline size_t desc_bytes(int ndiff, int nreif, int nrows, int nterms, int ndec,
                                             int nbrows, int nbslots)
{
    return align16(sizeof(int4) * (size_t)nrows) + align16(sizeof(int2) * (size_t)ndiff) +
           align16(sizeof(int2) * (size_t)nreif) + align16(sizeof(uint32_t) * (size_t)nterms) +
           align16(sizeof(int32_t) * (size_t)ndec) + align16(sizeof(int2) * (size_t)nbrows) +
           align16(sizeof(uint32_t) * (size_t)nbslots);
}

// View over global memory.
// A pointer every lane holds the same value of, kept in scalar registers.
template <typename T>
__device__ __forceinline__ const T *uptr(const T *p)
{
    const unsigned long long u = reinterpret_cast<unsigned long long>(p);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)u);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(u >> 32));
    return reinterpret_cast<const T *>(((unsigned long long)hi << 32) | lo);
}

__device__ inline View<false> view_global(const DevModel &m)
{
    View<false> v;
    v.nvars = m.nvars; v.ndiff = m.ndiff; v.nreif = m.nreif; v.nrows = m.nrows;
    v.nterms = m.nterms; v.ndec = m.ndec; v.objective = m.objective;
    v.row_group = m.row_group; v.row_chunks = m.row_chunks;
    v.nbrows = m.nbrows; v.bgroup = m.bgroup; v.bchunks = m.bchunks; v.nbterms = m.nbterms;
    v.diff_ = uptr(m.diff); v.reif_ = uptr(m.reif); v.rows_ = uptr(m.rows);
    v.terms_ = uptr(m.terms); v.dec_ = uptr(m.dec);
    v.brows_ = uptr(m.brows); v.bterms_ = uptr(m.bterms);
    v.adjp_ = uptr(m.adj_ptr); v.adj_ = uptr(m.adj);
    v.ncmd = m.ncmd;
    v.cmds_ = uptr(m.cmds); v.ccnt_ = uptr(m.ccnt); v.cent_ = uptr(m.cent);
    return v;
}

// Copy the descriptor tables into LDS at `dst` (all threads) and return a
// view over the copy.  Caller puts a barrier before the view is used.
__device__ inline View<true> stage_descriptors(const DevModel &m, char *dst)
{
    const int tid = threadIdx.x, W = blockDim.x;
    View<true> v;
    v.nvars = m.nvars; v.ndiff = m.ndiff; v.nreif = m.nreif; v.nrows = m.nrows;
    v.nterms = m.nterms; v.ndec = m.ndec; v.objective = m.objective;
    v.row_group = m.row_group; v.row_chunks = m.row_chunks;
    v.nbrows = m.nbrows; v.bgroup = m.bgroup; v.bchunks = m.bchunks; v.nbterms = m.nbterms;
    const int nbslots = m.nbrows * m.bgroup * m.bchunks;
    char *p = dst;
    int4 *rows = reinterpret_cast<int4 *>(p);
    p += align16(sizeof(int4) * (size_t)m.nrows);
    int2 *diff = reinterpret_cast<int2 *>(p);
    p += align16(sizeof(int2) * (size_t)m.ndiff);
    int2 *reif = reinterpret_cast<int2 *>(p);
    p += align16(sizeof(int2) * (size_t)m.nreif);
    uint32_t *terms = reinterpret_cast<uint32_t *>(p);
    p += align16(sizeof(uint32_t) * (size_t)m.nterms);
    int32_t *dec = reinterpret_cast<int32_t *>(p);
    p += align16(sizeof(int32_t) * (size_t)m.ndec);
    int2 *brows = reinterpret_cast<int2 *>(p);
    p += align16(sizeof(int2) * (size_t)m.nbrows);
    uint32_t *bterms = reinterpret_cast<uint32_t *>(p);
    for (int i = tid; i < m.nbrows; i += W) brows[i] = gread(m.brows + i);
    for (int i = tid; i < nbslots; i += W) bterms[i] = gread(m.bterms + i);
    for (int i = tid; i < m.nrows; i += W) rows[i] = gread(m.rows + i);
    for (int i = tid; i < m.ndiff; i += W) diff[i] = gread(m.diff + i);
    for (int i = tid; i < m.nreif; i += W) reif[i] = gread(m.reif + i);
    for (int i = tid; i < m.nterms; i += W) terms[i] = gread(m.terms + i);
    for (int i = tid; i < m.ndec; i += W) dec[i] = gread(m.dec + i);
    v.rows_ = rows; v.diff_ = diff; v.reif_ = reif; v.terms_ = terms; v.dec_ = dec;
    v.brows_ = brows; v.bterms_ = bterms;
    v.adjp_ = uptr(m.adj_ptr); v.adj_ = uptr(m.adj);
    v.ncmd = m.ncmd;
    v.cmds_ = uptr(m.cmds); v.ccnt_ = uptr(m.ccnt); v.cent_ = uptr(m.cent);
    return v;
}

// ------------------------------------------------------ propagation loop
// A sweep runs every item of one list per kind once.  A list is either the
// whole table of the kind (`in` = nullptr: entry t is descriptor t) or an
// LDS array of descriptor indices.  Wavefront w takes the entries
// 64 w + lane + k W, U chunks of 64 at a time: the loads of a chunk are all
// issued before any is used, and a chunk that lies wholly past the end of
// the list is skipped by the whole wavefront, so a sweep costs in proportion
// to the list's length.
//
// Entailed propagators.  A propagator is entailed in a store when none of
// its tells can tighten that store or any tighter one (its guards and bounds
// are monotone in the store).  Dropping it from the sweeps of every node
// below the one where that holds changes no fixed point (§3 Theorem 2: the
// fixed point is the least store closed under the remaining propagators,
// and the dropped ones are closed on every store that can follow).  With
// `out` set, a sweep also appends to `out` (in any order) each item it ran
// and did not find entailed, judged on the bounds it read joined with its
// own tells (a store no tighter than any later one), and counts them in
// *cnt; a row sweep also adds the terms of the rows it keeps to *tcnt.
struct ListIO {
    const uint16_t *in;   // nullptr: the whole table
    int n;                // entries to run
    uint16_t *out;        // compaction target, or nullptr
    int32_t *cnt;         // count of the kept entries
    int32_t *tcnt;        // rows: terms of the kept rows
};

// Append, per wavefront, the entries whose `keep` is set (U chunks) to out.
template <int U>
__device__ __forceinline__ void compact(const ListIO &io, const bool (&keep)[U], const int (&idx)[U])
{
    const int lane = threadIdx.x & 63;
    unsigned long long mk[U];
    int tot = 0;
#pragma unroll
    for (int u = 0; u < U; ++u) {
        mk[u] = __ballot(keep[u]);
        tot += __popcll(mk[u]);
    }
    if (tot == 0) return;
    int pos = 0;
    if (lane == 0)
        pos = __hip_atomic_fetch_add(io.cnt, tot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    pos = __builtin_amdgcn_readfirstlane(pos);
#pragma unroll
    for (int u = 0; u < U; ++u) {
        if (keep[u]) {
            const int r = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mk[u] >> 32),
                                                        __builtin_amdgcn_mbcnt_lo((uint32_t)mk[u], 0u));
            io.out[pos + r] = (uint16_t)idx[u];
        }
        pos += __popcll(mk[u]);
    }
}

// ------------------------------------------- dependency-driven propagation
// A propagator has to run again only after a bound it reads was tightened
// (chaotic iteration reaches the same least fixed point, §3 Theorem 2, as
// long as no propagator whose input changed is left out).  With marks on,
// every tell also sets its variable's bit in the sweep's change bitmap of
// that bound (lm / um); between sweeps the bitmaps are expanded through the
// variable -> propagator adjacency into the next sweep's work lists.
//
// The trail.  With trail_on, the first tell of a node on a variable also
// pushes the variable's (lb, ub) as the lane read it onto the workgroup's
// trail, so that a backtrack can restore the parent's store instead of
// recomputing it.  The value pushed is the one before the node: every tell
// is issued after its lane's test-and-set of the variable's trail bit (tm),
// LDS operations of a wavefront execute in issue order, and the lane that
// wins the bit read the variable before its own test-and-set, so before any
// tell of the node (each of which follows a losing or winning test-and-set
// that came later).
struct Dep {
    uint32_t *lm, *um;        // bounds tightened in this sweep (lb / ub)
    uint32_t *tm;             // variables already on this node's trail
    uint32_t *qm;             // propagators already on the next work lists
    uint16_t *wl;             // work lists: kind k at wl + woff[k], wcap[k] entries
    int4 *trail;              // this workgroup's trail (global), tcap entries
    int32_t *ttop;            // LDS word: entries pushed (may pass tcap)
    uint32_t *jobs;           // two-phase expansion: changed variables, jcap entries
    int32_t *jcnt;            // LDS word: entries in jobs (may pass jcap)
    int jcap;                 // 0: one-phase expansion
    int vshift, vmask, vw, qw;
    int woff[kDepKinds], wcap[kDepKinds], qoff[kDepKinds];
    int tcap;
    bool trail_on;
};

__device__ __forceinline__ void trail_push(const Dep &dp, int x, int2 rd)
{
    const int pos = __hip_atomic_fetch_add(dp.ttop, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    if (pos < dp.tcap) gwrite4(dp.trail + pos, make_int4(x, rd.x, rd.y, 0));
}

// tell lb(x) >= v (or ub(x) <= v) with marks: rd = (lb, ub) of x as the lane
// read it before deciding to tell
template <bool MK, bool LB>
__device__ __forceinline__ void tell_m(const Store st, const Dep &dp, int x, int32_t v, int2 rd)
{
    if constexpr (MK) {
        const uint32_t w = (uint32_t)x & (uint32_t)dp.vmask, bit = 1u << ((uint32_t)x >> dp.vshift);
        uint32_t old = bit;
        if (dp.trail_on)
            old = __hip_atomic_fetch_or(dp.tm + w, bit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        __builtin_amdgcn_sched_barrier(0);
        if (LB) tell_lb(st, x, v); else tell_ub(st, x, v);
        __hip_atomic_fetch_or((LB ? dp.lm : dp.um) + w, bit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (!(old & bit)) trail_push(dp, x, rd);
    } else {
        if (LB) tell_lb(st, x, v); else tell_ub(st, x, v);
    }
}

// Sum over the `G` lanes of a row group (G = 4, 8 or 16; groups are aligned
// so that every DPP source lane is in the same group).
__device__ __forceinline__ int group_sum(int x, int G)
{
    x += __builtin_amdgcn_update_dpp(0, x, 0xB1, 0xF, 0xF, false);   // quad_perm 1,0,3,2
    x += __builtin_amdgcn_update_dpp(0, x, 0x4E, 0xF, 0xF, false);   // quad_perm 2,3,0,1
    if (G >= 8) x += __builtin_amdgcn_update_dpp(0, x, 0x141, 0xF, 0xF, false);  // row_half_mirror
    if (G >= 16) x += __builtin_amdgcn_update_dpp(0, x, 0x140, 0xF, 0xF, false); // row_mirror
    return x;
}

// kind 1: x - y <= c  =>  ub(x) <= c + ub(y),  lb(y) >= lb(x) - c;
// entailed once ub(x) - lb(y) <= c.
template <bool DL, bool MK = false>
__device__ __forceinline__ void sweep_diff(const View<DL> &v, const Store st, const ListIO &io,
                                           const Dep &dp, bool &chg, bool &bad, uint32_t &nat)
{
    constexpr int U = 2;
    const int tid = threadIdx.x, lane = tid & 63, W = blockDim.x, n = io.n;
    // wavefronts take the chunks in reverse order: the reified items that
    // follow leave their last chunk to the first wavefronts, so the small
    // table of difference rows evens out the work per wavefront
    const int wrev = (W >> 6) - 1 - (tid >> 6);
    for (int c0 = uni(wrev * 64); c0 < n; c0 += U * W) {
        int idx[U];
        bool ok[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int t = c0 + u * W + lane;
            ok[u] = t < n;
            const int tc = ok[u] ? t : n - 1;
            idx[u] = io.in ? (int)io.in[tc] : tc;
        }
        int2 e[U], dx[U], dy[U];
#pragma unroll
        for (int u = 0; u < U; ++u)
            e[u] = c0 + u * W < n ? v.diff(idx[u]) : make_int2(0, 0x3fffffff);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            dx[u] = make_int2(0, 0);
            dy[u] = make_int2(0, 0);
            if (c0 + u * W < n) {
                dx[u] = dom(st, e[u].x & 0xffff);
                dy[u] = dom(st, (uint32_t)e[u].x >> 16);
            }
        }
        bool pu[U], pl[U], any = false;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int c = e[u].y;
            pu[u] = ok[u] && c + dy[u].y < dx[u].y;
            pl[u] = ok[u] && dx[u].x - c > dy[u].x;
            any |= pu[u] | pl[u];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) nat += lanes(pu[u]) + lanes(pl[u]);
        if (any) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int x = e[u].x & 0xffff, y = (uint32_t)e[u].x >> 16, c = e[u].y;
                const int nu = c + dy[u].y, nl = dx[u].x - c;
                if (pu[u]) { tell_m<MK, false>(st, dp, x, nu, dx[u]); chg = true; bad |= nu < dx[u].x; }
                if (pl[u]) { tell_m<MK, true>(st, dp, y, nl, dy[u]); chg = true; bad |= nl > dy[u].y; }
            }
        }
        if (io.out) {
            bool keep[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int c = e[u].y;
                const int ux = min(dx[u].y, c + dy[u].y), ly = max(dy[u].x, dx[u].x - c);
                keep[u] = ok[u] && ux - ly > c;
            }
            compact<U>(io, keep, idx);
        }
    }
}

// kind 2: b <=> (si <= sj and sj < si + d): the four guarded processes of
// [[phi <=> psi]] with interval entailment (see pccp.h).  The guarded
// tells on the start variables are merged per bound: each of ub(si),
// lb(sj), ub(sj), lb(si) gets the tightest value any enabled guard tells,
//   b true  : ub(si) <= ub(sj),    lb(sj) >= lb(si),
//             ub(sj) <= ub(si)+d-1, lb(si) >= lb(sj)-d+1
//   b false, si <= sj entailed   : lb(sj) >= lb(si)+d, ub(si) <= ub(sj)-d
//   b false, sj < si+d entailed  : ub(sj) <= ub(si)-1, lb(si) >= lb(sj)+1
// and is told only if that value is tighter than the bound read.
// Entailed once b = 1 with both conjuncts entailed, or b = 0 with one of
// them disentailed (lb(si) > ub(sj), or lb(sj) >= ub(si) + d).
template <bool DL, int U, bool MK = false>
__device__ __forceinline__ void sweep_reif(const View<DL> &v, const Store st, const ListIO &io,
                                           const Dep &dp, bool &chg, bool &bad, uint32_t &nat)
{
    const int tid = threadIdx.x, lane = tid & 63, W = blockDim.x, n = io.n;
    for (int c0 = uni(tid - lane); c0 < n; c0 += U * W) {
        int idx[U];
        bool ok[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int t = c0 + u * W + lane;
            ok[u] = t < n;
            const int tc = ok[u] ? t : n - 1;
            idx[u] = io.in ? (int)io.in[tc] : tc;
        }
        int2 e[U], di[U], dj[U], db[U];
#pragma unroll
        for (int u = 0; u < U; ++u)
            e[u] = c0 + u * W < n ? v.reif(idx[u]) : make_int2(0, 0);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            db[u] = di[u] = dj[u] = make_int2(0, 0);
            if (c0 + u * W < n) {
                db[u] = dom(st, e[u].x & 0xffff);
                di[u] = dom(st, (uint32_t)e[u].x >> 16);
                dj[u] = dom(st, e[u].y & 0xffff);
            }
        }
        bool keep[U] = {};
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int d = e[u].y >> 16;
            const int lbi = di[u].x, ubi = di[u].y, lbj = dj[u].x, ubj = dj[u].y;
            const int lbb = db[u].x, ubb = db[u].y;
            // With X = ub(sj) - lb(si) and Y = lb(sj) - ub(si): si <= sj is
            // entailed iff Y >= 0 and disentailed iff X < 0; sj < si + d is
            // entailed iff X < d and disentailed iff Y >= d.
            const int X = ubj - lbi, Y = lbj - ubi;
            const bool E1 = Y >= 0, E2 = X < d;
            const bool on = lbb >= 1, off = ubb <= 0;
            const bool t_b1 = !on && E1 && E2;           // psi entailed: b >= 1
            const bool t_b0 = !off && (X < 0 || Y >= d); // not psi: b <= 0
            // b = 1 tells both conjuncts; b = 0 tells the negation of the
            // conjunct that is not entailed: with si <= sj entailed,
            // sj >= si + d (d1 = d); with sj < si + d entailed, sj < si (d2 = 0)
            const bool a1 = on || (off && E1);           // ub(si), lb(sj)
            const bool a2 = on || (off && E2);           // ub(sj), lb(si)
            const int d1 = off ? d : 0, d2 = on ? d : 0;
            const int nui = ubj - d1, nlj = lbi + d1;
            const int nuj = ubi + d2 - 1, nli = lbj - d2 + 1;
            const bool p_ui = a1 && nui < ubi, p_lj = a1 && nlj > lbj;
            const bool p_uj = a2 && nuj < ubj, p_li = a2 && nli > lbi;
            if (io.out) {
                const int ui = p_ui ? nui : ubi, lj = p_lj ? nlj : lbj;
                const int uj = p_uj ? nuj : ubj, li = p_li ? nli : lbi;
                const bool b1 = on || t_b1, b0 = off || t_b0;
                const bool ent = (b1 && ui <= lj && uj <= li + d - 1) ||
                                 (b0 && (li > uj || lj >= ui + d));
                keep[u] = ok[u] && !ent;
            }
            nat += lanes(ok[u] && t_b1) + lanes(ok[u] && t_b0) + lanes(ok[u] && p_ui) +
                   lanes(ok[u] && p_lj) + lanes(ok[u] && p_uj) + lanes(ok[u] && p_li);
            if (!ok[u] || !(t_b1 | t_b0 | p_ui | p_lj | p_uj | p_li))
                continue;
            const int b = e[u].x & 0xffff, i = (uint32_t)e[u].x >> 16, j = e[u].y & 0xffff;
            chg = true;
            if (t_b1) { tell_m<MK, true>(st, dp, b, 1, db[u]); bad |= ubb < 1; }
            if (t_b0) { tell_m<MK, false>(st, dp, b, 0, db[u]); bad |= lbb > 0; }
            if (p_ui) { tell_m<MK, false>(st, dp, i, nui, di[u]); bad |= nui < lbi; }
            if (p_lj) { tell_m<MK, true>(st, dp, j, nlj, dj[u]); bad |= nlj > ubj; }
            if (p_uj) { tell_m<MK, false>(st, dp, j, nuj, dj[u]); bad |= nuj < lbj; }
            if (p_li) { tell_m<MK, true>(st, dp, i, nli, di[u]); bad |= nli > ubi; }
        }
        if (io.out) compact<U>(io, keep, idx);
    }
}

// One term's tell of  a x <= rr  (rr = rhs - (S - m_t)) given the bounds the
// lane read for x: is it tighter, and the new bound.  Division only for
// |a| > 1 (floor toward -inf for a > 0, ceil toward +inf for a < 0).
__device__ __forceinline__ bool term_tight(int a, int lbx, int ubx, int rhs, int S)
{
    return a > 0 ? rhs - (S - a * lbx) < a * ubx : rhs - (S - a * ubx) < a * lbx;
}

template <bool MK = false>
__device__ __forceinline__ void term_tell(const Store st, const Dep &dp, int x, int a, int lbx, int ubx,
                                          int rhs, int S, bool &chg, bool &bad)
{
    if (a > 0) {
        const int rr = rhs - (S - a * lbx);                 // a x <= rr
        const int nb = a == 1 ? rr : floor_div_pos(rr, a);
        tell_m<MK, false>(st, dp, x, nb, make_int2(lbx, ubx)); chg = true; bad |= nb < lbx;
    } else {
        const int rr = rhs - (S - a * ubx);                 // x >= ceil(rr / a)
        const int nb = a == -1 ? -rr : -floor_div_pos(rr, -a);
        tell_m<MK, true>(st, dp, x, nb, make_int2(lbx, ubx)); chg = true; bad |= nb > ubx;
    }
}

// kind 3: sum_t a_t x_t <= rhs.  A group of G lanes takes a row; lane l of
// the group holds terms first + l + G*k.  S (the sum of every term's
// smallest value, §2's lsum generalised) is a DPP sum over the group; each
// term is then told a_t x_t <= rhs - (S - m_t).  Rows are taken RR at a
// time per group; when every row fits in one chunk of TK terms per lane the
// tells use the bounds already in registers.  Entailed once the sum of the
// terms' largest values is at most rhs.
template <bool DL, int RR, bool MK = false>
__device__ __forceinline__ void sweep_rows(const View<DL> &v, const Store st, const ListIO &io,
                                           const Dep &dp, bool &chg, bool &bad, uint32_t &nat,
                                           uint32_t &nterm)
{
    constexpr int TK = 2;
    const int tid = threadIdx.x, W = blockDim.x, n = io.n;
    if (n == 0) return;
    const int G = v.row_group, gl = tid & (G - 1), gid = tid / G, NG = W / G;
    const int g0 = uni((tid & ~63) / G);     // first group of this wavefront
    const int KC = v.row_chunks;            // chunks of G terms in the longest row
    const bool cmp = io.out != nullptr;
    for (int rb0 = g0; rb0 < n; rb0 += RR * NG) {
        const int rbase = rb0 + (gid - g0);
        int ri[RR];
        int4 rd[RR];
        bool rok[RR];
#pragma unroll
        for (int q = 0; q < RR; ++q) {
            const int r = rbase + q * NG;
            rok[q] = r < n;
            const int rc = rok[q] ? r : n - 1;
            ri[q] = io.in ? (int)io.in[rc] : rc;
        }
#pragma unroll
        for (int q = 0; q < RR; ++q) rd[q] = v.rows(ri[q]);
#pragma unroll
        for (int q = 0; q < RR; ++q) nterm += rok[q] && gl == 0 ? (uint32_t)rd[q].y : 0u;
        int S[RR], Smax[RR];
        if (KC <= TK) {
            uint32_t tv[RR][TK];
            bool tok[RR][TK];
#pragma unroll
            for (int q = 0; q < RR; ++q)
#pragma unroll
                for (int k = 0; k < TK; ++k) {
                    const int o = gl + k * G;
                    tok[q][k] = rok[q] && o < rd[q].y;
                    tv[q][k] = v.terms(rd[q].x + (o < rd[q].y ? o : 0));
                }
            int2 td[RR][TK];
#pragma unroll
            for (int q = 0; q < RR; ++q)
#pragma unroll
                for (int k = 0; k < TK; ++k) td[q][k] = dom(st, tv[q][k] & 0xffff);
#pragma unroll
            for (int q = 0; q < RR; ++q) {
                int part = 0, pmax = 0;
#pragma unroll
                for (int k = 0; k < TK; ++k) {
                    const int a = (int32_t)tv[q][k] >> 16;
                    part += tok[q][k] ? (a > 0 ? a * td[q][k].x : a * td[q][k].y) : 0;
                    pmax += tok[q][k] ? (a > 0 ? a * td[q][k].y : a * td[q][k].x) : 0;
                }
                S[q] = group_sum(part, G);
                Smax[q] = cmp ? group_sum(pmax, G) : 0;
            }
            bool tight[RR][TK], any = false;
#pragma unroll
            for (int q = 0; q < RR; ++q)
#pragma unroll
                for (int k = 0; k < TK; ++k) {
                    tight[q][k] = tok[q][k] && term_tight((int32_t)tv[q][k] >> 16, td[q][k].x,
                                                          td[q][k].y, rd[q].z, S[q]);
                    any |= tight[q][k];
                    nat += lanes(tight[q][k]);
                }
            if (any) {
#pragma unroll
                for (int q = 0; q < RR; ++q)
#pragma unroll
                    for (int k = 0; k < TK; ++k)
                        if (tight[q][k])
                            term_tell<MK>(st, dp, tv[q][k] & 0xffff, (int32_t)tv[q][k] >> 16,
                                          td[q][k].x, td[q][k].y, rd[q].z, S[q], chg, bad);
            }
        } else {
            // long rows: sum chunk by chunk, then tell chunk by chunk
#pragma unroll
            for (int q = 0; q < RR; ++q) S[q] = Smax[q] = 0;
            for (int k = 0; k < KC; ++k) {
                const int o = gl + k * G;
#pragma unroll
                for (int q = 0; q < RR; ++q) {
                    if (rok[q] && o < rd[q].y) {
                        const uint32_t t = v.terms(rd[q].x + o);
                        const int a = (int32_t)t >> 16;
                        const int2 dx = dom(st, t & 0xffff);
                        S[q] += a > 0 ? a * dx.x : a * dx.y;
                        Smax[q] += a > 0 ? a * dx.y : a * dx.x;
                    }
                }
            }
#pragma unroll
            for (int q = 0; q < RR; ++q) {
                S[q] = group_sum(S[q], G);
                if (cmp) Smax[q] = group_sum(Smax[q], G);
            }
            for (int k = 0; k < KC; ++k) {
                const int o = gl + k * G;
#pragma unroll
                for (int q = 0; q < RR; ++q) {
                    const bool in = rok[q] && o < rd[q].y;
                    uint32_t t = 0;
                    int2 dx = make_int2(0, 0);
                    if (in) {
                        t = v.terms(rd[q].x + o);
                        // a bound re-read here can only have tightened since S
                        // was formed: the tell is then weaker, never unsound
                        dx = dom(st, t & 0xffff);
                    }
                    const int x = t & 0xffff, a = (int32_t)t >> 16;
                    const bool tt = in && term_tight(a, dx.x, dx.y, rd[q].z, S[q]);
                    nat += lanes(tt);
                    if (tt) term_tell<MK>(st, dp, x, a, dx.x, dx.y, rd[q].z, S[q], chg, bad);
                }
            }
        }
        if (cmp) {
            bool keep[RR];
#pragma unroll
            for (int q = 0; q < RR; ++q) keep[q] = rok[q] && gl == 0 && Smax[q] > rd[q].z;
            compact<RR>(io, keep, ri);
#pragma unroll
            for (int q = 0; q < RR; ++q)
                if (keep[q])
                    __hip_atomic_fetch_add(io.tcnt, rd[q].y, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_WORKGROUP);
        }
    }
}

// kind 4: sum_t a_t b_t <= rhs with every b_t in [0, 1] and a_t > 0.  This is
// kind 3's rule on 0/1 domains: with S = the sum of a_t over the terms with
// lb(b_t) = 1 and slack = rhs - S, a negative slack empties some term's
// interval (failure), and otherwise every open term (lb = 0 < ub) with
// a_t > slack is told ub(b_t) <= 0; no other tell of kind 3 tightens a 0/1
// store.  Products become selects and there is no division.  A group of G
// lanes takes a row; the terms of row r sit at r * G * KC + lane + G * k, so
// their addresses do not wait for the row descriptor; unused slots hold
// a = 0.  Entailed once the sum of a_t over the terms with ub(b_t) = 1 is at
// most rhs.
template <bool DL, int RB, bool MK = false>
__device__ __forceinline__ void sweep_brows(const View<DL> &v, const Store st, const ListIO &io,
                                            const Dep &dp, bool &chg, bool &bad, uint32_t &nat,
                                            uint32_t &nterm)
{
    constexpr int TB = 4;                   // term slots per lane held in registers
    const int tid = threadIdx.x, W = blockDim.x, n = io.n;
    if (n == 0) return;
    const int G = v.bgroup, gl = tid & (G - 1), gid = tid / G, NG = W / G;
    const int g0 = uni((tid & ~63) / G);     // first group of this wavefront
    const int KC = v.bchunks, SL = G * KC;
    const bool cmp = io.out != nullptr;
    for (int rb0 = g0; rb0 < n; rb0 += RB * NG) {
        const int rbase = rb0 + (gid - g0);
        int ri[RB];
        bool rok[RB];
#pragma unroll
        for (int q = 0; q < RB; ++q) {
            const int r = rbase + q * NG;
            rok[q] = r < n;
            const int rc = rok[q] ? r : n - 1;
            ri[q] = io.in ? (int)io.in[rc] : rc;
        }
        int2 rd[RB];
        int S[RB], Smax[RB];
        if (KC <= TB) {
            uint32_t tv[RB][TB];
#pragma unroll
            for (int q = 0; q < RB; ++q)
#pragma unroll
                for (int k = 0; k < TB; ++k)
                    tv[q][k] = k < KC ? v.bterms(ri[q] * SL + gl + k * G) : 0u;
#pragma unroll
            for (int q = 0; q < RB; ++q) rd[q] = v.brows(ri[q]);
#pragma unroll
            for (int q = 0; q < RB; ++q) nterm += rok[q] && gl == 0 ? (uint32_t)rd[q].y : 0u;
            // per slot only a (open term) or 0 (fixed term) survives the sums;
            // products with a 0/1 bound are 24-bit multiply-adds (a store
            // where a bound left [0, 1] has already failed)
            int rv[RB][TB];
#pragma unroll
            for (int q = 0; q < RB; ++q) {
                int part = 0, pmax = 0;
#pragma unroll
                for (int k = 0; k < TB; ++k) {
                    const int2 d = k < KC ? dom(st, tv[q][k] & 0xffff) : make_int2(0, 0);
                    const uint32_t a = tv[q][k] >> 16;
                    part = (int)__umul24(a, (uint32_t)d.x) + part;
                    pmax = (int)__umul24(a, (uint32_t)d.y) + pmax;
                    rv[q][k] = d.x < d.y ? (int)a : 0;
                }
                S[q] = group_sum(part, G);
                Smax[q] = cmp ? group_sum(pmax, G) : 0;
            }
            uint32_t tight = 0;
#pragma unroll
            for (int q = 0; q < RB; ++q) {
                const int slack = rd[q].x - S[q];
                if (rok[q] && slack < 0) { bad = true; chg = true; }
#pragma unroll
                for (int k = 0; k < TB; ++k)
                    tight |= (rok[q] && slack >= 0 && rv[q][k] > slack) ? 1u << (q * TB + k) : 0u;
            }
#pragma unroll
            for (int i = 0; i < RB * TB; ++i) nat += lanes((tight >> i) & 1u);
            if (__any(tight != 0)) {
#pragma unroll
                for (int q = 0; q < RB; ++q)
#pragma unroll
                    for (int k = 0; k < TB; ++k)
                        if (tight & (1u << (q * TB + k))) {
                            // an open term of a 0/1 variable reads (0, 1)
                            tell_m<MK, false>(st, dp, tv[q][k] & 0xffff, 0, make_int2(0, 1));
                            chg = true;
                        }
            }
        } else {
            // long rows: sum chunk by chunk, then tell chunk by chunk
#pragma unroll
            for (int q = 0; q < RB; ++q) {
                rd[q] = v.brows(ri[q]);
                S[q] = Smax[q] = 0;
                nterm += rok[q] && gl == 0 ? (uint32_t)rd[q].y : 0u;
            }
            for (int k = 0; k < KC; ++k) {
#pragma unroll
                for (int q = 0; q < RB; ++q) {
                    const uint32_t t = v.bterms(ri[q] * SL + gl + k * G);
                    const int a = (int)(t >> 16);
                    const int2 dx = dom(st, t & 0xffff);
                    S[q] += dx.x > 0 ? a : 0;
                    Smax[q] += dx.y > 0 ? a : 0;
                }
            }
#pragma unroll
            for (int q = 0; q < RB; ++q) {
                S[q] = group_sum(S[q], G);
                if (cmp) Smax[q] = group_sum(Smax[q], G);
                if (rok[q] && rd[q].x - S[q] < 0) { bad = true; chg = true; }
            }
            for (int k = 0; k < KC; ++k) {
#pragma unroll
                for (int q = 0; q < RB; ++q) {
                    const uint32_t t = v.bterms(ri[q] * SL + gl + k * G);
                    const int a = (int)(t >> 16);
                    // a bound re-read here can only have tightened since S was
                    // formed: an open term is still told soundly
                    const int2 dx = dom(st, t & 0xffff);
                    const bool tt = rok[q] && a > 0 && a > rd[q].x - S[q] && dx.x < dx.y;
                    nat += lanes(tt);
                    if (tt) {
                        tell_m<MK, false>(st, dp, t & 0xffff, 0, dx);
                        chg = true;
                        bad |= dx.x > 0;
                    }
                }
            }
        }
        if (cmp) {
            bool keep[RB];
#pragma unroll
            for (int q = 0; q < RB; ++q) keep[q] = rok[q] && gl == 0 && Smax[q] > rd[q].x;
            compact<RB>(io, keep, ri);
#pragma unroll
            for (int q = 0; q < RB; ++q)
                if (keep[q])
                    __hip_atomic_fetch_add(io.tcnt, rd[q].y, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_WORKGROUP);
        }
    }
}

// kind 5: guarded commands {g_1, ..., g_n} => x <- f (§3, guarded normal
// form; §2, ask and tell).  One lane per command: the guards are entailment
// tests on single bounds (lb(y) >= c or ub(y) <= c); when all hold, f =
// k + sum_t a_t y_t is formed from the bounds that keep it monotone (for a
// lower-bound tell: lb(y) when a > 0, ub(y) when a < 0; the opposite for an
// upper-bound tell), divided by div with rounding toward the sound side
// (ceil for lb, floor for ub), and joined into the target bound if tighter.
// The model is validated so that |k| + sum |a_t| max |bound(y_t)| < 2^30:
// f cannot overflow int32 on a store that has not failed.  Commands are not
// compacted into item lists; they run whole-table in the every-table and
// item-list modes, and from their work list in the dependency-driven mode.
template <bool DL, bool MK = false>
__device__ __forceinline__ void sweep_cmd(const View<DL> &v, const Store st, const ListIO &io,
                                          const Dep &dp, bool &chg, bool &bad, uint32_t &nat)
{
    const int tid = threadIdx.x, lane = tid & 63, W = blockDim.x, n = io.n;
    for (int c0 = uni(tid - lane); c0 < n; c0 += W) {
        const int t = c0 + lane;
        bool fire = false, lbt = false;
        int x = 0, nb = 0;
        int2 dx = make_int2(0, 0);
        if (t < n) {
            const int q = io.in ? (int)io.in[t] : t;
            const int4 c = v.cmd(q);
            const uint32_t cn = v.ccnt(q);
            const int ng = (int)(cn & 0xffffu), nt = (int)(cn >> 16), e0 = c.w;
            bool hold = true;
            for (int g = 0; g < ng && hold; ++g) {
                const int2 e = v.cent(e0 + g);
                const int2 d = dom(st, e.x & 0xffff);
                hold = ((e.x >> 16) & 1) ? d.y <= e.y : d.x >= e.y;
            }
            if (hold) {
                int f = c.y;
                for (int u = 0; u < nt; ++u) {
                    const int2 e = v.cent(e0 + ng + u);
                    const int2 d = dom(st, e.x & 0xffff);
                    f += e.y * (((e.x >> 16) & 1) ? d.y : d.x);
                }
                x = c.x & 0xffff;
                lbt = ((c.x >> 16) & 1) == 0;
                const int div = c.z;
                dx = dom(st, x);
                if (lbt) {
                    nb = div == 1 ? f : -floor_div_pos(-f, div);
                    fire = nb > dx.x;
                } else {
                    nb = div == 1 ? f : floor_div_pos(f, div);
                    fire = nb < dx.y;
                }
            }
        }
        nat += lanes(fire);
        if (fire) {
            chg = true;
            if (lbt) {
                tell_m<MK, true>(st, dp, x, nb, dx);
                bad |= nb > dx.y;
            } else {
                tell_m<MK, false>(st, dp, x, nb, dx);
                bad |= nb < dx.x;
            }
        }
    }
}

// The item lists of one node, per kind (0 difference rows, 1 reified items,
// 2 linear rows, 3 Boolean rows): the first sweep runs in[k] (nin[k]
// entries; nullptr = the whole table; tin = terms of the rows in in[2] and
// in[3]) and, when out[0] is set, writes the items it keeps to out[k] with
// their counts in cnt[k] and the kept rows' terms in cnt[4]; later sweeps
// run the kept lists.
constexpr int kKinds = 4;
constexpr int kKindsDep = kDepKinds;
constexpr int kDepSetWords = kDepKinds;  // per set: the kinds' list lengths
constexpr int kListWords = kKinds + 1;
// Item lists (the live mode) and work lists (the dependency-driven mode) are
// never used together; each must stay clear of the words every mode uses.
static_assert(C_CNT + 3 * kListWords <= C_SKIP, "item-list counts overlap C_SKIP");
static_assert(C_DCNT + 2 * kDepSetWords <= C_DTERMS && C_DTERMS < C_TTOP,
              "work-list counts overlap the term count or the trail words");
static_assert(C_TTOP != C_SKIP && C_TTOP != C_JCNT && C_TTOP != C_MAXW && C_TTOP != C_ATOM &&
                  C_THI != C_SKIP && C_THI != C_JCNT && C_THI != C_MAXW && C_THI != C_ATOM &&
                  C_THI < 32 && C_THI >= C_DCNT + 2 * kDepSetWords,
              "the trail words need words of their own in the dependency-driven mode");
static_assert(C_MAXW >= C_CNT + 3 * kListWords && C_MAXW != C_SKIP && C_MAXW != C_JCNT &&
                  C_MAXW < 32, "the stack word must lie outside every count range");
static_assert(C_ATOM >= C_CNT + 3 * kListWords && C_ATOM != C_SKIP && C_ATOM != C_JCNT &&
                  C_ATOM != C_MAXW && C_ATOM < 32, "the join counter needs a word of its own");
struct NodeLists {
    const uint16_t *in[kKinds];
    int nin[kKinds];
    int tin;
    uint16_t *out[kKinds];
    int32_t *cnt;
};

// Fixed point of the LDS store `st` under the propagators of the lists `L`.
// Returns 1 if the loop saw a failure, 0 at a fixed point (the post scan
// still has to look for an empty interval the loop did not see).  ex[] gets
// the items run per kind and the row terms visited.
// Precondition: a barrier separates this call from any earlier read of the
// control words C_FLAG*, C_POSTFAIL, C_KEY and of the out lists.
// LIVE: L may carry lists.  LEAN: fewer items per lane per chunk (for the
// lists' compaction, and for the high-occupancy search kernel).
template <bool DL, bool LIVE, bool LEAN = LIVE>
__device__ __forceinline__ int propagate_wg(const View<DL> &v, const Store st, int32_t *ctl, const NodeLists &L,
                            uint32_t &nsweeps, unsigned long long (&ex)[4], uint32_t &nat)
{
    const int tid = threadIdx.x, lane = tid & 63;
    const bool cmp = L.out[0] != nullptr;
    if (tid == 0) {
        ctl[C_FLAG0] = 0;
        ctl[C_FLAG1] = 0;
        ctl[C_FLAG2] = 0;
        ctl[C_POSTFAIL] = 0;
        *reinterpret_cast<unsigned long long *>(ctl + C_KEY) = ~0ull;
        if (cmp)
            for (int k = 0; k < kListWords; ++k) L.cnt[k] = 0;
    }
    lds_barrier();
    int32_t *tc = cmp ? L.cnt + kKinds : nullptr;
    ListIO d{L.in[0], L.nin[0], L.out[0], cmp ? L.cnt : nullptr, nullptr};
    ListIO r{L.in[1], L.nin[1], L.out[1], cmp ? L.cnt + 1 : nullptr, nullptr};
    ListIO w{L.in[2], L.nin[2], L.out[2], cmp ? L.cnt + 2 : nullptr, tc};
    ListIO b{L.in[3], L.nin[3], L.out[3], cmp ? L.cnt + 3 : nullptr, tc};
    int terms = L.tin;
    int slot = 0;
    const Dep nodep{};
    for (;;) {
        bool chg = false, bad = false;
        sweep_diff(v, st, d, nodep, chg, bad, nat);
        sweep_reif<DL, LEAN ? 2 : 4>(v, st, r, nodep, chg, bad, nat);
        uint32_t unused_terms = 0;   // the tables' term counts are known
        sweep_rows<DL, LEAN ? 2 : 4>(v, st, w, nodep, chg, bad, nat, unused_terms);
        sweep_brows<DL, LEAN ? 1 : 2>(v, st, b, nodep, chg, bad, nat, unused_terms);
        if (v.ncmd) sweep_cmd(v, st, ListIO{nullptr, v.ncmd, nullptr, nullptr, nullptr}, nodep, chg, bad, nat);
        ex[0] += (unsigned)d.n;
        ex[1] += (unsigned)r.n;
        ex[2] += (unsigned)(w.n + b.n + v.ncmd);
        ex[3] += (unsigned)terms;
        const int flags = (__any(chg) ? 1 : 0) | (__any(bad) ? 2 : 0);
        if (lane == 0 && flags)
            __hip_atomic_fetch_or(&ctl[slot], flags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        const int next = slot == 2 ? 0 : slot + 1;
        if (tid == 0)
            ctl[next] = 0;
        lds_barrier();
        ++nsweeps;
        const int f = lds_ld(&ctl[slot]);
        if (f & 2) return 1;
        if (!(f & 1)) return 0;
        slot = next;
        if (d.out) {
            // after the first sweep: run what it kept
            d = ListIO{d.out, uni(lds_ld(&L.cnt[0])), nullptr, nullptr, nullptr};
            r = ListIO{r.out, uni(lds_ld(&L.cnt[1])), nullptr, nullptr, nullptr};
            w = ListIO{w.out, uni(lds_ld(&L.cnt[2])), nullptr, nullptr, nullptr};
            b = ListIO{b.out, uni(lds_ld(&L.cnt[3])), nullptr, nullptr, nullptr};
            terms = uni(lds_ld(&L.cnt[kKinds]));
        }
    }
}

// Work lists of the next sweep from the change bitmaps of the last one:
// every propagator that reads a tightened bound (rows once: the queued bit
// qm of a row is set when it is listed; see dep_queue).  Clears the bitmaps.
// cnt: list counts of the 5 kinds, zeroed by the caller before a barrier.
// A count past its list's capacity means the next sweep runs that kind's
// whole table.
// Bitmap word w is read by wavefront w % nw, so the variables of one
// region of the store (the start times, say) spread over all wavefronts.
// one chunk of adjacency entries (0 = none): queue the propagators that read
// a bound in `reads`
__device__ __forceinline__ void dep_queue(const Dep &dp, int32_t *cnt, uint32_t e, uint32_t reads)
{
    const int lane = threadIdx.x & 63;
    const int k = (int)((e >> 16) & 7u), idx = (int)(e & 0xffffu);
    bool fire = (e & reads) != 0;
    // difference rows, reified items and guarded commands may be listed
    // twice (two of their variables changed): running one twice costs less
    // than the queued bit's round trip; rows, which visit many terms, are
    // listed once
    if (fire && (k == 2 || k == 3)) {
        const int p = idx + (k == 2 ? dp.qoff[2] : dp.qoff[3]);
        const uint32_t qb = 1u << (p & 31);
        fire = !(__hip_atomic_fetch_or(dp.qm + (p >> 5), qb, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_WORKGROUP) & qb);
    }
#pragma unroll
    for (int kk = 0; kk < kKindsDep; ++kk) {
        const unsigned long long mk = __ballot(fire && k == kk);
        if (mk == 0) continue;
        int pos = 0;
        if (lane == 0)
            pos = __hip_atomic_fetch_add(cnt + kk, __popcll(mk), __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_WORKGROUP);
        pos = __builtin_amdgcn_readfirstlane(pos);
        if (fire && k == kk) {
            const int r = pos + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mk >> 32),
                                                              __builtin_amdgcn_mbcnt_lo((uint32_t)mk, 0u));
            if (r < dp.wcap[kk]) dp.wl[dp.woff[kk] + r] = (uint16_t)idx;
        }
    }
}

// Inclusive prefix sum over the 64 lanes of a wavefront (every lane
// active) with DPP moves: shifts by 1, 2, 4 and 8 within each row of 16
// lanes, then the broadcast of lane 15 of a row into the next row (kept by
// rows 1 and 3) and of lane 31 into rows 2 and 3.
__device__ __forceinline__ int wave_incl_sum(int x)
{
    const int lane = threadIdx.x & 63, rl = lane & 15;
    int t = __builtin_amdgcn_mov_dpp(x, 0x111, 0xf, 0xf, false);    // row_shr:1
    if (rl >= 1) x += t;
    t = __builtin_amdgcn_mov_dpp(x, 0x112, 0xf, 0xf, false);        // row_shr:2
    if (rl >= 2) x += t;
    t = __builtin_amdgcn_mov_dpp(x, 0x114, 0xf, 0xf, false);        // row_shr:4
    if (rl >= 4) x += t;
    t = __builtin_amdgcn_mov_dpp(x, 0x118, 0xf, 0xf, false);        // row_shr:8
    if (rl >= 8) x += t;
    t = __builtin_amdgcn_mov_dpp(x, 0x142, 0xf, 0xf, false);        // row_bcast:15
    if ((lane & 31) >= 16) x += t;
    t = __builtin_amdgcn_mov_dpp(x, 0x143, 0xf, 0xf, false);        // row_bcast:31
    if (lane >= 32) x += t;
    return x;
}

// One-phase expansion: each wavefront takes the bitmap words w with
// w % nw == its index (64 words a round, one per lane).  The changed
// variables of a round are taken in batches of one per lane (the lowest
// bit left in the lane's word): every lane loads its variable's adjacency
// range at once, a prefix sum over the lanes lays the batch's entries end
// to end, and the wavefront queues them 64 at a time.  A batch of
// variables with few readers each (a Boolean is read by its reified item
// and its rows) thus costs one round trip for the ranges and one per 64
// entries, instead of two per variable.
template <bool DL>
__device__ __forceinline__ void dep_expand(const View<DL> &v, const Dep &dp, int32_t *cnt)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
    for (int base = 0; base < dp.vw; base += 64 * nw) {
        const int w = base + wid + nw * lane;
        uint32_t bl = 0, bu = 0;
        if (w < dp.vw) {
            bl = dp.lm[w];
            bu = dp.um[w];
            if (bl | bu) {
                dp.lm[w] = 0;
                dp.um[w] = 0;
            }
        }
        uint32_t bits = bl | bu;
        while (__ballot(bits != 0)) {
            int a0 = 0, n = 0;
            uint32_t reads = 0;
            if (bits) {
                const int b = __builtin_ctz(bits);
                bits &= bits - 1;
                const int x = (b << dp.vshift) | w;
                reads = (((bl >> b) & 1u) ? kAdjLb : 0u) | (((bu >> b) & 1u) ? kAdjUb : 0u);
                a0 = v.adjp(x);
                n = v.adjp(x + 1) - a0;
            }
            // lane i's entries take positions [excl, incl) of the batch
            const int incl = wave_incl_sum(n);
            const int excl = incl - n;
            const int total = __builtin_amdgcn_readlane(incl, 63);
            const unsigned long long has = __ballot(n > 0);
            for (int lo = 0; lo < total; lo += 64) {
                const int g = lo + lane;
                // the lanes whose ranges meet [lo, lo + 64): entry g is the
                // one whose range holds it (the load stays inside that range)
                unsigned long long meet = has & __ballot(excl < lo + 64) & __ballot(incl > lo);
                int off = 0;
                uint32_t rd = 0;
                bool hit = false;
                while (meet) {
                    const int L = __builtin_ctzll(meet);
                    meet &= meet - 1;
                    const int se = __builtin_amdgcn_readlane(excl, L);
                    const int sn = __builtin_amdgcn_readlane(n, L);
                    if (g >= se && g - se < sn) {
                        hit = true;
                        off = __builtin_amdgcn_readlane(a0, L) + (g - se);
                        rd = (uint32_t)__builtin_amdgcn_readlane((int)reads, L);
                    }
                }
                dep_queue(dp, cnt, hit ? v.adj(off) : 0u, rd);
            }
        }
    }
}

// Two-phase expansion for workgroups of many wavefronts, where one
// wavefront's share of the changed variables (a start time of a large
// instance is read by hundreds of propagators) would keep the others
// waiting.  Phase 1 (before a barrier): each bitmap word's owner lane clears
// it and appends its variables, with the bounds that changed, to the job
// list.  Phase 2 (`dep_expand_jobs`, after the barrier): every wavefront
// loads the adjacency ranges of 64 listed variables at a time, numbers
// their chunks of 64 entries in list order and takes chunks wid, wid + nw,
// ...  A list longer than jcap makes the next sweep run every table.
__device__ __forceinline__ void dep_expand_list(const Dep &dp)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
    for (int base = 0; base < dp.vw; base += 64 * nw) {
        const int w = base + wid + nw * lane;
        if (w >= dp.vw) continue;
        const uint32_t bl = dp.lm[w], bu = dp.um[w];
        uint32_t bits = bl | bu;
        if (!bits) continue;
        dp.lm[w] = 0;
        dp.um[w] = 0;
        int pos = __hip_atomic_fetch_add(dp.jcnt, __popc(bits), __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_WORKGROUP);
        while (bits) {
            const int b = __builtin_ctz(bits);
            bits &= bits - 1;
            if (pos < dp.jcap)
                dp.jobs[pos] = (uint32_t)((b << dp.vshift) | w) | (((bl >> b) & 1u) << 30) |
                               (((bu >> b) & 1u) << 31);
            ++pos;
        }
    }
}

template <bool DL>
__device__ __forceinline__ void dep_expand_jobs(const View<DL> &v, const Dep &dp, int32_t *cnt)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const int n = uni(lds_ld(dp.jcnt));
    if (n > dp.jcap) {
        // too many changed variables: every table next sweep
        if (threadIdx.x == 0)
            for (int k = 0; k < kDepKinds; ++k) cnt[k] = dp.wcap[k] + 1;
        return;
    }
    for (int r0 = 0; r0 < n; r0 += 64) {
        const int i = r0 + lane;
        uint32_t ent = 0;
        int a0 = 0, a1 = 0;
        if (i < n) {
            ent = dp.jobs[i];
            const int x = (int)(ent & 0x3fffffffu);
            a0 = v.adjp(x);
            a1 = v.adjp(x + 1);
        }
        const int nch = (a1 - a0 + 63) >> 6;
        // inclusive scan of the chunk counts over the wavefront
        int incl = nch;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int t = __shfl_up(incl, d, 64);
            if (lane >= d) incl += t;
        }
        const int first = incl - nch;
        const int total = __shfl(incl, 63, 64);
        for (int j = wid; j < total; j += nw) {
            // the variable whose chunks contain j: the last lane starting at or before j
            const int L = 63 - __builtin_clzll(__ballot(first <= j && nch > 0));
            const int b0 = __shfl(a0, L, 64), b1 = __shfl(a1, L, 64);
            const uint32_t e0 = (uint32_t)__shfl((int)ent, L, 64);
            const uint32_t reads = ((e0 >> 30) & 1u ? kAdjLb : 0u) | ((e0 >> 31) & 1u ? kAdjUb : 0u);
            const int a = b0 + 64 * (j - __shfl(first, L, 64));
            dep_queue(dp, cnt, a + lane < b1 ? v.adj(a + lane) : 0u, reads);
        }
    }
}

// Fixed point of `st` with dependency-driven sweeps.  full: the first sweep
// runs every table (the store is new: a subtree root or a recomputed node;
// marks left by an earlier node are cleared); otherwise the store is a
// fixed point joined with the tells marked since (a decision, the objective
// bound), and the first sweep runs what they make ready.  Returns as
// propagate_wg; ex[0..2] count the items run, and the terms of the rows run
// are summed into ctl[C_DTERMS] (complete after the caller's next barrier).
// TWO: the build may run the two-phase expansion (workgroups of 8 or more
// wavefronts, dp.jcap > 0); the high-occupancy build never does.
template <bool DL, bool LEAN, bool TWO>
__device__ __forceinline__ int propagate_dep(const View<DL> &v, const Store st, int32_t *ctl, const Dep &dp, bool full,
                             uint32_t &nsweeps, unsigned long long (&ex)[4], uint32_t &nat)
{
    const int tid = threadIdx.x, lane = tid & 63, W = blockDim.x;
    if (tid == 0) {
        ctl[C_FLAG0] = 0;
        ctl[C_FLAG1] = 0;
        ctl[C_FLAG2] = 0;
        ctl[C_POSTFAIL] = 0;
        *reinterpret_cast<unsigned long long *>(ctl + C_KEY) = ~0ull;
        for (int k = 0; k < 2 * kDepSetWords; ++k) ctl[C_DCNT + k] = 0;
        ctl[C_JCNT] = 0;
        ctl[C_DTERMS] = 0;
    }
    if (full)
        for (int w = tid; w < dp.vw; w += W) {
            dp.lm[w] = 0;
            dp.um[w] = 0;
            dp.tm[w] = 0;
        }
    lds_barrier();
    int set = 0;   // count set of the lists the next sweep runs
    // one expansion into the count set cs, ending with a barrier
    auto expand = [&](int32_t *cs) {
        if (TWO && dp.jcap) {
            dep_expand_list(dp);
            lds_barrier();
            dep_expand_jobs(v, dp, cs);
        } else {
            dep_expand(v, dp, cs);
        }
        lds_barrier();
    };
    if (!full) expand(ctl + C_DCNT);
    const int tab[kDepKinds] = {v.ndiff, v.nreif, v.nrows, v.nbrows, v.ncmd};
    int slot = 0;
    bool all = full;
    uint32_t nterm = 0;   // terms of the rows this lane's groups ran
    // every wavefront's term count into ctl[C_DTERMS] (read after a barrier)
    auto publish_terms = [&]() {
        uint32_t t = nterm;
#pragma unroll
        for (int d = 32; d > 0; d >>= 1) t += (uint32_t)__shfl_xor((int)t, d, 64);
        if (lane == 0 && t)
            __hip_atomic_fetch_add(&ctl[C_DTERMS], (int32_t)t, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_WORKGROUP);
    };
    for (;;) {
        const int32_t *c = ctl + C_DCNT + kDepSetWords * set;
        ListIO io[kDepKinds];
        bool whole[kDepKinds];
#pragma unroll
        for (int k = 0; k < kDepKinds; ++k) {
            const int n = all ? 0 : uni(lds_ld(&c[k]));
            whole[k] = all || n > dp.wcap[k];
            io[k] = whole[k] ? ListIO{nullptr, tab[k], nullptr, nullptr, nullptr}
                             : ListIO{dp.wl + dp.woff[k], n, nullptr, nullptr, nullptr};
        }
        if (tid == 0) {
            for (int k = 0; k < kDepSetWords; ++k) ctl[C_DCNT + kDepSetWords * (set ^ 1) + k] = 0;
            ctl[C_JCNT] = 0;    // read by the last expansion before the barrier ending it
        }
        // the queued bits of the lists run now are cleared for the next expansion
        for (int w = tid; w < dp.qw; w += W) dp.qm[w] = 0;
        bool chg = false, bad = false;
        sweep_diff<DL, true>(v, st, io[0], dp, chg, bad, nat);
        sweep_reif<DL, LEAN ? 2 : 4, true>(v, st, io[1], dp, chg, bad, nat);
        sweep_rows<DL, LEAN ? 2 : 4, true>(v, st, io[2], dp, chg, bad, nat, nterm);
        sweep_brows<DL, LEAN ? 1 : 2, true>(v, st, io[3], dp, chg, bad, nat, nterm);
        if (io[4].n) sweep_cmd<DL, true>(v, st, io[4], dp, chg, bad, nat);
        ex[0] += (unsigned)io[0].n;
        ex[1] += (unsigned)io[1].n;
        ex[2] += (unsigned)(io[2].n + io[3].n + io[4].n);
        const int flags = (__any(chg) ? 1 : 0) | (__any(bad) ? 2 : 0);
        if (lane == 0 && flags)
            __hip_atomic_fetch_or(&ctl[slot], flags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        const int next = slot == 2 ? 0 : slot + 1;
        if (tid == 0)
            ctl[next] = 0;
        lds_barrier();
        ++nsweeps;
        const int f = lds_ld(&ctl[slot]);
        if (f & 2) {
            // marks of the failed sweep: the next node starts from a store
            // where none of them applies
            for (int w = tid; w < dp.vw; w += W) {
                dp.lm[w] = 0;
                dp.um[w] = 0;
            }
            publish_terms();
            return 1;
        }
        if (!(f & 1)) {
            publish_terms();
            return 0;
        }
        slot = next;
        set ^= 1;
        all = false;
        expand(ctl + C_DCNT + kDepSetWords * set);
    }
}

// ------------------------------------------------------ store copies
// A store occupies store_bytes(nI, nvars) bytes: pairs rounded up to an even
// count (the padding pair holds (0, 0)), then the Boolean words rounded up
// to a multiple of four (padding bytes 0: the open interval [0, 1]); so the
// whole store is a whole number of 16-byte blocks and neither padding reads
// as empty.

// Does some interval of the store (every lane's share) read as empty?
__device__ __forceinline__ bool store_failed(const Store st, int nvars)
{
    const int tid = threadIdx.x, W = blockDim.x;
    bool bad = false;
    const int np = store_pairs(st.nI) >> 1;            // two pairs per 16 bytes
    const int4 *s4 = reinterpret_cast<const int4 *>(st.p);
    for (int q = tid; q < np; q += W) {
        const int4 a = s4[q];
        bad |= (a.x > a.y) | (a.z > a.w);
    }
    const int nb = store_bool_words(st.nI, nvars) >> 2;  // four words per 16 bytes
    const uint4 *b4 = reinterpret_cast<const uint4 *>(st.b);
    for (int q = tid; q < nb; q += W) {
        const uint4 w = b4[q];
        bad |= (((w.x & (w.x >> 1)) | (w.y & (w.y >> 1)) | (w.z & (w.z >> 1)) |
                 (w.w & (w.w >> 1))) & 0x01010101u) != 0u;
    }
    return bad;
}

// st <- the box (lb, ub) of global arrays; with `orig`, store variable x
// reads entry orig[x] (the model's numbering), else entry x
__device__ __forceinline__ void load_box(const Store st, const int32_t *lb0, const int32_t *ub0,
                                         int nvars, const int32_t *orig = nullptr)
{
    const int tid = threadIdx.x, W = blockDim.x, nIp = store_pairs(st.nI);
    for (int x = tid; x < nIp; x += W) {
        const int i = x < st.nI ? (orig ? gread(orig + x) : x) : 0;
        st.p[x] = x < st.nI ? make_int2(gread(lb0 + i), gread(ub0 + i)) : make_int2(0, 0);
    }
    const int nw = store_bool_words(st.nI, nvars);
    for (int w = tid; w < nw; w += W) {
        uint32_t word = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int x = st.nI + 4 * w + k;
            if (x < nvars) {
                const int i = orig ? gread(orig + x) : x;
                word |= bool_bits(gread(lb0 + i), gread(ub0 + i)) << (8 * k);
            }
        }
        st.b[w] = word;
    }
}

// write the store to global arrays (entry orig[x] for store variable x)
__device__ __forceinline__ void store_box(const Store st, int32_t *lb, int32_t *ub, int nvars,
                                          const int32_t *orig)
{
    const int tid = threadIdx.x, W = blockDim.x;
    for (int x = tid; x < nvars; x += W) {
        const int2 d = dom(st, x);
        const int i = gread(orig + x);
        gwrite(lb + i, d.x);
        gwrite(ub + i, d.y);
    }
}

// copy a whole store (bytes of the same layout) from src to dst;
// SG/DG: source/destination in global memory (else LDS)
template <bool SG, bool DG>
__device__ __forceinline__ void copy_store(char *dst, const char *src, int nI, int nvars)
{
    const int tid = threadIdx.x, W = blockDim.x, nq = (int)(store_bytes(nI, nvars) >> 4);
    const int4 *s4 = reinterpret_cast<const int4 *>(src);
    int4 *d4 = reinterpret_cast<int4 *>(dst);
    for (int q = tid; q < nq; q += W) {
        const int4 a = SG ? gread(s4 + q) : s4[q];
        if (DG) gwrite4(d4 + q, a); else d4[q] = a;
    }
}

// ------------------------------------------------------ learned branching
// Features of decision variable q in the store (lb, ub) (x = dec[q], initial
// interval [lo, hi], H = max(1, hi - lo)):
//   f0 = (lb(x) - lo)/H, f1 = (ub(x) - lo)/H, f2 = (ub(x) - lb(x))/H,
//   f3 = degree share, f4 = min(1, min over rows x - y <= c of
//   (c + ub(y) - lb(x))/H), f5 = static load + (#reified items with si = x
//   and lb(b) >= 1) / N.
// The learned-branching tables are read through the instance's DevModel
// (global memory), so the propagation view stays small.
template <bool DL>
__device__ __forceinline__ void candidate_features(const View<DL> &v, const DevModel *m, int q,
                                                   const Store st, float f[kNumFeat])
{
    const int x = v.dec(q);
    const float *fs = m->fstat + 8 * (size_t)q;
    const int lo = __float_as_int(gread_f(fs + 0));
    const float invH = gread_f(fs + 1), degn = gread_f(fs + 2), sl = gread_f(fs + 3);
    const float invN = gread_f(fs + 4);
    const int2 dx = dom(st, x);
    const int lbx = dx.x, ubx = dx.y;
    f[0] = (float)(lbx - lo) * invH;
    f[1] = (float)(ubx - lo) * invH;
    f[2] = (float)(ubx - lbx) * invH;
    f[3] = degn;
    float slack = 1.0f;
    const int r1 = gread(m->fr_ptr + q + 1);
    for (int k = gread(m->fr_ptr + q); k < r1; ++k) {
        const int2 e = gread(m->fr + k);
        slack = fminf(slack, (float)(e.y + dom(st, e.x).y - lbx) * invH);
    }
    f[4] = slack;
    int cnt = 0;
    const int b1 = gread(m->fb_ptr + q + 1);
    for (int k = gread(m->fb_ptr + q); k < b1; ++k)
        cnt += dom(st, gread(m->fb + k)).x >= 1;
    f[5] = sl + (float)cnt * invN;
}

// bf16 -> fp32
__device__ __forceinline__ float bf16f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// One lane per hidden unit: lane k of every wave holds W1[k][.], b1[k], w2[k].
struct MlpLane {
    float w1[kNumFeat];
    float b1, w2;
};

__device__ inline MlpLane load_mlp_lane(const uint16_t *p)
{
    MlpLane ml;
    const int k = threadIdx.x & 63;
#pragma unroll
    for (int f = 0; f < kNumFeat; ++f) ml.w1[f] = p ? bf16f(p[k * kNumFeat + f]) : 0.f;
    ml.b1 = p ? bf16f(p[kHidden * kNumFeat + k]) : 0.f;
    ml.w2 = p ? bf16f(p[kHidden * kNumFeat + kHidden + k]) : 0.f;
    return ml;
}

// Sum over the 64 lanes in a fixed order (DPP within rows of 16, then the
// four row sums in lane order); every lane gets the total.
__device__ __forceinline__ float wave_sum_f(float x)
{
    x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0xB1, 0xF, 0xF, false));
    x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x4E, 0xF, 0xF, false));
    x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x141, 0xF, 0xF, false));
    x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x140, 0xF, 0xF, false));
    const float r0 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 0));
    const float r1 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 16));
    const float r2 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 32));
    const float r3 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 48));
    return ((r0 + r1) + r2) + r3;
}

// Branching key of score s for candidate q: the smallest key is the largest
// score, ties to the smallest q.
__device__ __forceinline__ unsigned long long score_key(float s, int q)
{
    const uint32_t u = __float_as_uint(s);
    const uint32_t asc = (u & 0x80000000u) ? ~u : (u | 0x80000000u);
    return ((unsigned long long)(~asc) << 32) | (uint32_t)q;
}

// After the loop: look for an empty interval anywhere in the store and, if
// `branch` is set, find the branching variable (smallest key among unfixed
// decision variables).  Ends with a barrier; results in ctl[C_POSTFAIL] and
// the 64-bit word at ctl[C_KEY] (~0 when every decision variable is fixed).
// The store is 16-byte aligned and padded to a multiple of 4 variables;
// the pad holds (0, 0).
// With branching 2 (learned), `fsc` is an LDS scratch of 8 floats per
// decision variable and `ml` the lane's slice of the network.
template <bool DL>
__device__ __forceinline__ void post_scan(const View<DL> &v, const Store st, int32_t *ctl,
                          int branching, bool branch, float *fsc = nullptr,
                          const uint16_t *mlp = nullptr, const DevModel *m = nullptr)
{
    const int tid = threadIdx.x, W = blockDim.x, lane = tid & 63;
    bool bad = store_failed(st, v.nvars);
    unsigned long long key = ~0ull;
    if (branch && branching == 2) {
        // features of every unfixed candidate into LDS ...
        for (int q = tid; q < v.ndec; q += W) {
            const int2 dx = dom(st, v.dec(q));
            const bool open = dx.y > dx.x;
            fsc[8 * q + 6] = open ? 1.f : 0.f;
            if (open) {
                float f[kNumFeat];
                candidate_features(v, m, q, st, f);
#pragma unroll
                for (int k = 0; k < kNumFeat; ++k) fsc[8 * q + k] = f[k];
            }
        }
        lds_barrier();
        // ... then one wave per candidate, one lane per hidden unit
        const MlpLane ml = load_mlp_lane(mlp);
        const int wid = tid >> 6, nw = W >> 6;
        for (int q = wid; q < v.ndec; q += nw) {
            if (fsc[8 * q + 6] == 0.f) continue;
            float z = ml.b1;
#pragma unroll
            for (int k = 0; k < kNumFeat; ++k) z = fmaf(ml.w1[k], fsc[8 * q + k], z);
            const float sc = wave_sum_f(ml.w2 * fmaxf(z, 0.f));
            const unsigned long long k2 = score_key(sc, q);
            key = k2 < key ? k2 : key;
        }
    } else if (branch) {
        for (int q = tid; q < v.ndec; q += W) {
            const int2 dx = dom(st, v.dec(q));
            const int w = dx.y - dx.x;
            if (w > 0) {
                const unsigned long long k =
                    branching == 1 ? (unsigned long long)q
                                   : (((unsigned long long)(uint32_t)w << 32) | (uint32_t)q);
                key = k < key ? k : key;
            }
        }
        key = wave_min_u64(key);
    }
    if (__any(bad) && lane == 0)
        __hip_atomic_store(&ctl[C_POSTFAIL], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    if (branch && lane == 0 && key != ~0ull)
        __hip_atomic_fetch_min(reinterpret_cast<unsigned long long *>(ctl + C_KEY), key,
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    lds_barrier();
}

// apply decision word (var | side << 16, val) to the store as a join
__device__ __forceinline__ void apply_decision(const Store st, int2 dcs)
{
    const int x = dcs.x & 0xffff;
    if (dcs.x & kSideBit)
        tell_lb(st, x, dcs.y + 1);
    else
        tell_ub(st, x, dcs.y);
}

// ------------------------------------------------ features of given stores
// Features (6 floats per decision variable) of nbox stores, one workgroup
// per store: out[box][q][f].  The same device function the search uses.
__global__ __launch_bounds__(1024) void features_kernel(const DevModel *mp, int nbox,
                                                        const int32_t *lb_in, const int32_t *ub_in,
                                                        float *out)
{
    extern __shared__ __align__(16) char smem[];
    const DevModel m = *mp;
    const int tid = threadIdx.x, W = blockDim.x;
    const Store st = make_store(smem, m.nI);
    const View<false> v = view_global(m);
    for (int box = blockIdx.x; box < nbox; box += gridDim.x) {
        const size_t off = (size_t)box * m.nvars;
        load_box(st, lb_in + off, ub_in + off, m.nvars, m.vorig);
        lds_barrier();
        for (int q = tid; q < m.ndec; q += W) {
            float f[kNumFeat];
            candidate_features(v, mp, q, st, f);
            for (int k = 0; k < kNumFeat; ++k)
                out[((size_t)box * m.ndec + q) * kNumFeat + k] = f[k];
        }
        lds_barrier();
    }
}

hipError_t launch_features(const DevModel *m_dev, size_t store, int nbox, const int32_t *lb_in,
                           const int32_t *ub_in, float *out, hipStream_t stream)
{
    const size_t lds = store;
    const int grid = nbox < 2048 ? nbox : 2048;
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(features_kernel),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    (void)hipGetLastError();
    hipLaunchKernelGGL(features_kernel, dim3(grid), dim3(256), lds, stream, m_dev, nbox, lb_in,
                       ub_in, out);
    return hipGetLastError();
}

// ------------------------------------------------ batch of propagations
// One workgroup per box: fixed point of box k of instance `m`.
// lb_in/ub_in/lb_out/ub_out are [nbox][nvars]; status[k] = 0 fixpoint,
// 1 failed; sweeps[k] = sweeps of the loop (may be null).
template <bool DL>
__global__ __launch_bounds__(1024) void propagate_batch_kernel(
    const DevModel *mp, int nbox, const int32_t *lb_in, const int32_t *ub_in,
    int32_t *lb_out, int32_t *ub_out, int32_t *status, int32_t *sweeps)
{
    extern __shared__ __align__(16) char smem[];
    const DevModel m = *mp;
    const int tid = threadIdx.x;
    int32_t *ctl = reinterpret_cast<int32_t *>(smem);
    char *sb = reinterpret_cast<char *>(ctl + kCtlWords);
    const Store st = make_store(sb, m.nI);
    char *dsc = sb + store_bytes(m.nI, m.nvars);
    View<DL> v;
    if constexpr (DL) v = stage_descriptors(m, dsc); else v = view_global(m);
    const NodeLists L{{nullptr, nullptr, nullptr, nullptr}, {m.ndiff, m.nreif, m.nrows, m.nbrows},
                      m.nterms + m.nbterms, {nullptr, nullptr, nullptr, nullptr}, nullptr};
    for (int box = blockIdx.x; box < nbox; box += gridDim.x) {
        const size_t off = (size_t)box * m.nvars;
        load_box(st, lb_in + off, ub_in + off, m.nvars, m.vorig);
        uint32_t nsw = 0;
        unsigned long long ex[4] = {0, 0, 0, 0};
        lds_barrier();
        uint32_t nat = 0;
        const int rc = propagate_wg<DL, false>(v, st, ctl, L, nsw, ex, nat);
        post_scan(v, st, ctl, 0, false);
        const int failed = rc | lds_ld(&ctl[C_POSTFAIL]);
        store_box(st, lb_out + off, ub_out + off, m.nvars, m.vorig);
        if (tid == 0) {
            status[box] = failed;
            if (sweeps) sweeps[box] = (int32_t)nsw;
        }
        lds_barrier();
    }
}

// A tell by one thread outside the sweeps (a decision, the objective
// bound), with marks and, with dp.trail_on, the trail.
template <bool LB>
__device__ __forceinline__ void tell_one(const Store st, const Dep &dp, int x, int32_t v)
{
    const int2 d = dom(st, x);
    if (LB ? v <= d.x : v >= d.y) return;
    tell_m<true, LB>(st, dp, x, v, d);
}

// ------------------------------------------- incremental fixed points
// One workgroup per box.  The box is a fixed point of instance `m` joined
// with one decision on one variable; only the propagators that read a bound
// the decision tightened run in the first sweep, and each later sweep runs
// those that read a bound the one before tightened (dependency-driven
// propagation: a chaotic iteration that leaves out only propagators whose
// inputs did not change, so it reaches the same least fixed point, §3
// Theorem 2).  status[k]: 0 fixed point, 1 failed, -1 dvar[k] outside the
// store (the box is copied unchanged).
__global__ __launch_bounds__(1024) void propagate_incr_kernel(const DevModel *mp, IncrParams A)
{
    extern __shared__ __align__(16) char smem[];
    const DevModel m = *mp;
    const int tid = threadIdx.x, W = blockDim.x;
    int32_t *ctl = reinterpret_cast<int32_t *>(smem);
    char *sb = reinterpret_cast<char *>(ctl + kCtlWords);
    const Store st = make_store(sb, m.nI);
    char *p = sb + store_bytes(m.nI, m.nvars);
    const int vw = 1 << A.dep_vshift;
    Dep dp{};
    dp.lm = reinterpret_cast<uint32_t *>(p);
    dp.um = dp.lm + vw;
    dp.tm = dp.um + vw;
    p += align16(12 * (size_t)vw);
    dp.qm = reinterpret_cast<uint32_t *>(p);
    p += align16(4 * (size_t)A.dep_qw);
    dp.wl = reinterpret_cast<uint16_t *>(p);
    p += align16(2 * (size_t)(A.dep_wcap[0] + A.dep_wcap[1] + A.dep_wcap[2] + A.dep_wcap[3] +
                              A.dep_wcap[4]));
    dp.jobs = reinterpret_cast<uint32_t *>(p);
    dp.jcap = A.dep_jcap;
    dp.jcnt = ctl + C_JCNT;
    dp.vshift = A.dep_vshift;
    dp.vmask = vw - 1;
    dp.vw = vw;
    dp.qw = A.dep_qw;
    const int items[kDepKinds] = {m.ndiff, m.nreif, m.nrows, m.nbrows, m.ncmd};
    int wo = 0, qo = 0;
    for (int k = 0; k < kDepKinds; ++k) {
        dp.woff[k] = wo;
        dp.wcap[k] = A.dep_wcap[k];
        dp.qoff[k] = qo;
        wo += A.dep_wcap[k];
        qo += items[k];
    }
    dp.trail = nullptr;
    dp.tcap = 0;
    dp.ttop = ctl + C_TTOP;
    dp.trail_on = false;
    const View<false> v = view_global(m);
    for (int w = tid; w < dp.qw; w += W) dp.qm[w] = 0;
    for (int box = blockIdx.x; box < A.nbox; box += gridDim.x) {
        const size_t off = (size_t)box * m.nvars;
        load_box(st, A.lb_in + off, A.ub_in + off, m.nvars, m.vorig);
        for (int w = tid; w < 3 * vw; w += W) dp.lm[w] = 0;
        const int xo = gread(A.dvar + box);
        const bool valid = xo >= 0 && xo < m.nvars;
        const int x = valid ? gread(m.vnew + xo) : 0;
        lds_barrier();
        if (tid == 0 && valid) {
            // the decision: joins with marks, so the first sweep runs the
            // propagators that read the bounds it tightened
            tell_one<true>(st, dp, x, gread(A.dlo + box));
            tell_one<false>(st, dp, x, gread(A.dhi + box));
        }
        lds_barrier();
        uint32_t nsw = 0, nat = 0;
        unsigned long long ex[4] = {0, 0, 0, 0};
        int rc = 0;
        if (valid) rc = propagate_dep<false, true, true>(v, st, ctl, dp, false, nsw, ex, nat);
        post_scan(v, st, ctl, 0, false);
        const int failed = rc | lds_ld(&ctl[C_POSTFAIL]);
        store_box(st, A.lb_out + off, A.ub_out + off, m.nvars, m.vorig);
        if (tid == 0) {
            A.status[box] = valid ? failed : -1;
            if (A.sweeps) A.sweeps[box] = (int32_t)nsw;
        }
        lds_barrier();
    }
}

// ------------------------------------------------------------ the queue
// Bounded lock-free MPMC queue of subtree records (D. Vyukov's bounded
// queue: one sequence number per slot).  Only lane 0 of a workgroup calls
// these.
__device__ __forceinline__ long long q_claim_pop(const SearchParams &P)
{
    SearchGlobals *g = P.g;
    unsigned long long pos = g_load(&g->q_head);
    for (;;) {
        const unsigned long long seq = g_load_acq(&P.q_seq[pos % (unsigned)P.qcap]);
        const long long dif = (long long)(seq - (pos + 1));
        if (dif == 0) {
            if (g_cas(&g->q_head, pos, pos + 1))
                return (long long)pos;
        } else if (dif < 0) {
            return -1;
        } else {
            pos = g_load(&g->q_head);
        }
    }
}

__device__ __forceinline__ void q_release_slot(const SearchParams &P, unsigned long long pos)
{
    g_store_rel(&P.q_seq[pos % (unsigned)P.qcap], pos + (unsigned long long)P.qcap);
}

__device__ __forceinline__ long long q_claim_push(const SearchParams &P)
{
    SearchGlobals *g = P.g;
    unsigned long long pos = g_load(&g->q_tail);
    for (;;) {
        const unsigned long long seq = g_load_acq(&P.q_seq[pos % (unsigned)P.qcap]);
        const long long dif = (long long)(seq - pos);
        if (dif == 0) {
            if (g_cas(&g->q_tail, pos, pos + 1))
                return (long long)pos;
        } else if (dif < 0) {
            return -1;  // full
        } else {
            pos = g_load(&g->q_tail);
        }
    }
}

__device__ __forceinline__ void q_publish(const SearchParams &P, unsigned long long pos)
{
    g_store_rel(&P.q_seq[pos % (unsigned)P.qcap], pos + 1);
}

__device__ inline RecHdr *q_slot(const SearchParams &P, unsigned long long pos)
{
    return reinterpret_cast<RecHdr *>(P.q_data + (size_t)(pos % (unsigned)P.qcap) * P.slot_bytes);
}

// FNV-1a 64 over the little-endian bytes, finalised by MurmurHash3 fmix64.
template <bool DL>
__device__ __forceinline__ unsigned long long solution_hash(const Store st, const View<DL> &v, int n)
{
    unsigned long long h = 0xcbf29ce484222325ull;
    for (int i = 0; i < n; ++i) {
        const uint32_t val = (uint32_t)dom(st, v.dec(i)).x;
        for (int k = 0; k < 4; ++k) {
            h ^= (val >> (8 * k)) & 0xffu;
            h *= 0x100000001b3ull;
        }
    }
    h ^= h >> 33;
    h *= 0xff51afd7ed558ccdull;
    h ^= h >> 33;
    h *= 0xc4ceb9fe1a85ec53ull;
    h ^= h >> 33;
    return h;
}


// ------------------------------------------------------------ search
// The decision stack.  Level k of the path is {var | side << 16 |
// donated << 17, value, trail start of level k + 1, 0}; every level is kept
// in this workgroup's slice of global memory and the kRing deepest levels
// written are also kept in an LDS ring (slot k mod kRing), so that the LDS
// a workgroup needs does not grow with the stack capacity.  `maxw` (an LDS
// word) is the deepest level written since the subtree was taken: level k
// is in the ring while k > maxw - kRing, since only a write of a level
// k + j kRing (j >= 1) reuses its slot.  put() is called by one lane at a
// time; reads of global levels by other lanes follow a full barrier.
constexpr int kRing = 256;
struct Stack {
    int4 *ring;          // LDS, kRing entries
    int4 *g;             // global, max_depth entries
    int32_t *maxw;       // LDS word
    __device__ __forceinline__ bool in_ring(int k) const { return k > lds_ld(maxw) - kRing; }
    __device__ __forceinline__ int4 get(int k) const
    {
        return in_ring(k) ? ring[k & (kRing - 1)] : gread(g + k);
    }
    __device__ __forceinline__ void put(int k, int4 e) const
    {
        const int mw = lds_ld(maxw);
        if (k > mw) *maxw = k;
        if (k > mw - kRing) ring[k & (kRing - 1)] = e;
        gwrite4(g + k, e);
    }
};

// State only lane 0 uses lives in LDS (not in every lane's registers).
struct Lane0 {
    unsigned long long nodes, fails, sols, sweeps, don, maxd;
    unsigned long long since_flush, known_total, pf_qt, pf_qh;
    unsigned long long ex[4];     // items run per kind, row terms visited
    unsigned long long atom;      // lattice joins issued
    long long t_start;
    int32_t local_best, pf_best, pf_abort, pf_idle, idle_reg, pf_iabort;
};
static_assert(sizeof(Lane0) <= 4 * (kCtlWords - 32), "Lane0 must fit in the control block");

// lane 0: publish this workgroup's counters for instance `is`
__device__ __forceinline__ void flush_counters(Lane0 &z, InstState *is, int mode)
{
    g_add(&is->nodes, z.nodes);
    g_add(&is->fails, z.fails);
    g_add(&is->sweeps, z.sweeps);
    g_add(&is->donations, z.don);
    g_add(&is->pops, 1ull);
    for (int k = 0; k < 4; ++k) g_add(&is->ex[k], z.ex[k]);
    g_add(&is->atomics, z.atom);
    if (mode == 1) g_add(&is->solutions, z.sols);
    __hip_atomic_fetch_max(&is->max_depth, z.maxd, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    z.nodes = z.fails = z.sweeps = z.don = z.sols = z.maxd = 0;
    z.ex[0] = z.ex[1] = z.ex[2] = z.ex[3] = 0;
    z.atom = 0;
}

// Persistent kernel: every workgroup loops { take a subtree record; DFS it }
// until the queue is empty and no subtree is in progress, or a limit hits.
// LIVE: item lists (see propagate_wg) in three LDS buffers: R holds the
// items the subtree root kept, A and B alternate down the current path; a
// backtrack restarts from R, as the store restarts from the root's.
// HI: workgroups of at most 256 threads and at least 7 wavefronts per SIMD
// (at most 72 VGPRs; 6 and 80 with dependency-driven sweeps, whose extra
// state spills more at 72 and measured fastest at 6): more resident
// subproblems per CU to hide the latency of the dependent loads, with
// leaner unrolling.
#ifndef PCCP_HI_DEP_WAVES
#define PCCP_HI_DEP_WAVES 6
#endif
#ifndef PCCP_HI_WAVES
#define PCCP_HI_WAVES 7
#endif
template <bool DL, bool RL, bool LEARN, int PM, bool HI>
__global__ __launch_bounds__(HI ? 256 : 1024, HI ? (PM == 2 ? PCCP_HI_DEP_WAVES : PCCP_HI_WAVES) : 1) void search_kernel(SearchParams P)
{
    constexpr bool LIVE = PM == 1, DEP = PM == 2;
    extern __shared__ __align__(16) char smem[];
    const int tid = threadIdx.x, W = blockDim.x;
    const size_t SB = (size_t)P.max_store;    // bytes of the largest store of the launch
    int32_t *ctl = reinterpret_cast<int32_t *>(smem);
    Lane0 &z = *reinterpret_cast<Lane0 *>(ctl + 32);
    char *stb = reinterpret_cast<char *>(ctl + kCtlWords);   // the current store
    char *rstb;                                                // the subtree root's store
    char *p;
    if (RL) {
        rstb = stb + SB;
        p = rstb + SB;
    } else {
        rstb = P.root_scratch + (size_t)blockIdx.x * SB;
        p = stb + SB;
    }
    Store st = make_store(stb, 0);          // laid out for each instance taken
    const Stack stk{reinterpret_cast<int4 *>(p),
                    P.gstack + (size_t)blockIdx.x * (size_t)P.max_depth, ctl + C_MAXW};
    p += align16(sizeof(int4) * (size_t)kRing);
    float *fsc = reinterpret_cast<float *>(p);
    if (LEARN) p += align16(32 * (size_t)P.max_ndec);
    uint16_t *lbuf = reinterpret_cast<uint16_t *>(p);
    const int lcap = (int)(align16(2 * (size_t)(P.max_items[0] + P.max_items[1] + P.max_items[2] +
                                                P.max_items[3])) / 2);
    if (LIVE) p += 2 * 3 * (size_t)lcap;
    // dependency-driven propagation: the three variable bitmaps, the
    // propagator marks and the work lists
    Dep dp{};
    if (DEP) {
        const int vw = 1 << P.dep_vshift;
        dp.lm = reinterpret_cast<uint32_t *>(p);
        dp.um = dp.lm + vw;
        dp.tm = dp.um + vw;
        p += align16(12 * (size_t)vw);
        dp.qm = reinterpret_cast<uint32_t *>(p);
        p += align16(4 * (size_t)P.dep_qw);
        dp.wl = reinterpret_cast<uint16_t *>(p);
        p += align16(2 * (size_t)(P.dep_wcap[0] + P.dep_wcap[1] + P.dep_wcap[2] + P.dep_wcap[3] +
                                  P.dep_wcap[4]));
        dp.jobs = reinterpret_cast<uint32_t *>(p);
        p += align16(4 * (size_t)P.dep_jcap);
        dp.jcap = P.dep_jcap;
        dp.jcnt = ctl + C_JCNT;
        dp.vshift = P.dep_vshift;
        dp.vmask = vw - 1;
        dp.vw = vw;
        dp.qw = P.dep_qw;
        int wo = 0, qo = 0;
        for (int k = 0; k < kDepKinds; ++k) {
            dp.woff[k] = wo;
            dp.wcap[k] = P.dep_wcap[k];
            dp.qoff[k] = qo;
            wo += P.dep_wcap[k];
            qo += k < 4 ? P.max_items[k] : 0;
        }
        dp.trail = P.trail + (size_t)blockIdx.x * (size_t)P.tcap;
        dp.tcap = P.tcap;
        dp.ttop = ctl + C_TTOP;
        dp.trail_on = false;
        for (int w = tid; w < 3 * vw; w += W) dp.lm[w] = 0;
        for (int w = tid; w < P.dep_qw; w += W) dp.qm[w] = 0;
    }
    char *dsc = p;
    const int koff[kKinds] = {0, P.max_items[0], P.max_items[0] + P.max_items[1],
                              P.max_items[0] + P.max_items[1] + P.max_items[2]};
    const int branching = LEARN ? 2 : (P.branching == 1 ? 1 : 0);

    if (tid == 0) {
        z.nodes = z.fails = z.sols = z.sweeps = z.don = z.maxd = 0;
        z.ex[0] = z.ex[1] = z.ex[2] = z.ex[3] = 0;
        z.atom = 0;
        ctl[C_ATOM] = 0;
        z.since_flush = z.known_total = z.pf_qt = z.pf_qh = 0;
        z.t_start = g_load(&P.g->t_start);
        z.local_best = INT32_MAX;
        z.pf_best = INT32_MAX;
        z.pf_abort = z.pf_idle = z.idle_reg = 0;
    }
    int cur_inst = -1;
    View<DL> v{};

    for (;;) {
        // ---- take a record (lane 0)
        if (tid == 0) {
            long long got = -2;
            for (;;) {
                if (g_load(&P.g->abort) != 0) { got = -2; break; }
                const long long pos = q_claim_pop(P);
                if (pos >= 0) { got = pos; break; }
                if (g_load_acq(&P.g->outstanding) == 0) { got = -2; break; }
                if (P.t_limit_ticks > 0 && (long long)wall_clock64() - z.t_start > P.t_limit_ticks) {
                    g_store_rel(&P.g->abort, 2);
                    got = -2;
                    break;
                }
                if (!z.idle_reg) { g_add(&P.g->idle, 1); z.idle_reg = 1; }
                __builtin_amdgcn_s_sleep(8);
            }
            if (got >= 0 && z.idle_reg) { g_add(&P.g->idle, -1); z.idle_reg = 0; }
            ctl[C_SLOT] = (int32_t)(got & 0xffffffff);
            ctl[C_SLOT_HI] = (int32_t)(got >> 32);
            if (got >= 0) {
                const RecHdr *h = q_slot(P, (unsigned long long)got);
                ctl[C_INST] = h->inst;
                ctl[C_LEN] = h->len;
            }
            ctl[C_SKIP] = 0;
            if (got >= 0 && P.inst_node_limit > 0 && g_load(&P.inst[ctl[C_INST]].abandon) != 0) {
                // a subtree of an abandoned instance: drop it
                InstState *ai = &P.inst[ctl[C_INST]];
                q_release_slot(P, (unsigned long long)got);
                if (g_add(&ai->outstanding, -1) == 1)
                    __hip_atomic_store(&ai->t_done, (long long)wall_clock64(), __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
                g_add(&P.g->outstanding, -1);
                ctl[C_SKIP] = 1;
            }
        }
        full_barrier();
        const long long pos = (long long)(((unsigned long long)(uint32_t)uni(ctl[C_SLOT_HI]) << 32) |
                                          (uint32_t)uni(ctl[C_SLOT]));
        if (pos < 0)
            break;
        if (uni(ctl[C_SKIP])) {
            full_barrier();
            continue;
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        const int inst = uni(ctl[C_INST]);
        const int len = uni(ctl[C_LEN]);
        const int2 *rec = reinterpret_cast<const int2 *>(q_slot(P, (unsigned long long)pos) + 1);
        const DevModel &m = P.models[inst];
        if (inst != cur_inst) {
            if (tid == 0) z.local_best = INT32_MAX;
            if constexpr (DL) v = stage_descriptors(m, dsc); else v = view_global(m);
            st = make_store(stb, m.nI);
            cur_inst = inst;
        }
        const int nvars = m.nvars, ndec = m.ndec, objective = m.objective;
        load_box(st, m.lb0, m.ub0, nvars);
        lds_barrier();
        // the record's decisions: onto the stack (the deepest kRing also in
        // the ring) and into the store
        for (int i = tid; i < len; i += W) {
            const int2 dcs = gread(rec + i);
            const int4 e = make_int4(dcs.x & (0xffff | (int)kSideBit), dcs.y, 0, 0);
            gwrite4(stk.g + i, e);
            if (i >= len - kRing) stk.ring[i & (kRing - 1)] = e;
            apply_decision(st, make_int2(e.x, e.y));
        }
        if (tid == 0) ctl[C_MAXW] = len - 1;
        full_barrier();  // every lane is done reading the record
        if (tid == 0)
            q_release_slot(P, (unsigned long long)pos);

        const int depth0 = len;
        int depth = len;
        bool first = true;
        // DEP: the node's store is new (subtree root, recomputed node): the
        // first sweep runs every table and nothing goes on the trail
        bool node_full = true;
        if (DEP && tid == 0) {
            ctl[C_TTOP] = 0;
            ctl[C_THI] = depth0;
        }
        bool finished = false;
        // item lists: 0 = whole tables, 1 = R, 2 = A, 3 = B
        int in_sel = 0, out_sel = 1;
        InstState *is = &P.inst[inst];
        if (tid == 0) {
            z.pf_best = g_load(&is->best);
            z.pf_abort = 0;
            z.pf_iabort = 0;
        }
        bool abandoned = false;
        // ---- depth-first search of this subtree
        for (;;) {
            if (tid == 0) {
                int stop = z.pf_abort != 0 ? 1 : (z.pf_iabort != 0 ? 2 : 0);
                if (P.node_limit > 0 && z.known_total + z.since_flush >= (unsigned long long)P.node_limit) {
                    g_store_rel(&P.g->abort, 1);
                    stop = 1;
                }
                if (P.t_limit_ticks > 0 && (long long)wall_clock64() - z.t_start > P.t_limit_ticks) {
                    g_store_rel(&P.g->abort, 2);
                    stop = 1;
                }
                // the host word is read at system scope, past the device caches
                if (P.cancel && (z.since_flush & 255) == 0 &&
                    __hip_atomic_load(const_cast<int32_t *>(P.cancel), __ATOMIC_RELAXED,
                                      __HIP_MEMORY_SCOPE_SYSTEM) != 0) {
                    g_store_rel(&P.g->abort, 3);
                    stop = 1;
                }
                ctl[C_STOP] = stop;
                if (!stop && P.mode == 1) {
                    if (z.pf_best < z.local_best) z.local_best = z.pf_best;
                    if (z.local_best != INT32_MAX) {
                        if constexpr (DEP) {
                            dp.trail_on = !node_full;
                            tell_one<false>(st, dp, objective, z.local_best - 1);
                        } else {
                            tell_ub(st, objective, z.local_best - 1);
                        }
                    }
                }
                // loads consumed at the next node, so their latency overlaps
                // this node's propagation
                z.pf_best = g_load(&is->best);
                z.pf_abort = g_load(&P.g->abort);
                if (P.inst_node_limit > 0) z.pf_iabort = g_load(&is->abandon);
                if (P.donate) {
                    z.pf_idle = g_load(&P.g->idle);
                    z.pf_qt = g_load(&P.g->q_tail);
                    z.pf_qh = g_load(&P.g->q_head);
                }
            }
            lds_barrier();
            if (const int sv = uni(lds_ld(&ctl[C_STOP]))) {
                abandoned = sv == 2;
                break;
            }
            NodeLists L;
            if (LIVE && in_sel != 0) {
                const int32_t *c = ctl + C_CNT + kListWords * (in_sel - 1);
                uint16_t *b = lbuf + (size_t)(in_sel - 1) * lcap;
                for (int k = 0; k < kKinds; ++k) {
                    L.in[k] = b + koff[k];
                    L.nin[k] = uni(lds_ld(&c[k]));
                }
                L.tin = uni(lds_ld(&c[kKinds]));
            } else {
                for (int k = 0; k < kKinds; ++k) L.in[k] = nullptr;
                L.nin[0] = v.ndiff; L.nin[1] = v.nreif; L.nin[2] = v.nrows; L.nin[3] = v.nbrows;
                L.tin = v.nterms + v.nbterms;
            }
            if (LIVE) {
                uint16_t *b = lbuf + (size_t)(out_sel - 1) * lcap;
                for (int k = 0; k < kKinds; ++k) L.out[k] = b + koff[k];
                L.cnt = ctl + C_CNT + kListWords * (out_sel - 1);
            } else {
                for (int k = 0; k < kKinds; ++k) L.out[k] = nullptr;
                L.cnt = nullptr;
            }
            uint32_t nsw = 0, nat = 0;
            unsigned long long ex[4] = {0, 0, 0, 0};
            int rc;
            if constexpr (DEP) {
                dp.trail_on = !node_full;
                // work lists are short: lean unrolling (fewer registers)
                rc = propagate_dep<DL, true, !HI>(v, st, ctl, dp, node_full, nsw, ex, nat);
                // the next node's trail marks start empty; a node whose
                // changes did not all fit on the trail cannot be undone
                for (int w = tid; w < dp.vw; w += W) dp.tm[w] = 0;
                if (tid == 0 && !node_full && lds_ld(ctl + C_TTOP) > dp.tcap) ctl[C_THI] = depth;
            } else {
                rc = propagate_wg<DL, LIVE, LIVE || HI>(v, st, ctl, L, nsw, ex, nat);
            }
            // each wavefront's joins, read by lane 0 after the scan's barrier
            if ((tid & 63) == 0 && nat)
                __hip_atomic_fetch_add(ctl + C_ATOM, (int32_t)nat, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_WORKGROUP);
            post_scan(v, st, ctl, branching, rc == 0, fsc, P.mlp, &m);
            const int failed = uni(rc | lds_ld(&ctl[C_POSTFAIL]));
            const unsigned long long key =
                *reinterpret_cast<volatile unsigned long long *>(ctl + C_KEY);
            if (tid == 0) {
                z.nodes += 1;
                z.since_flush += 1;
                z.sweeps += nsw;
                for (int k = 0; k < 4; ++k) z.ex[k] += ex[k];
                if constexpr (DEP) z.ex[3] += (uint32_t)lds_ld(ctl + C_DTERMS);
                z.atom += (uint32_t)lds_ld(ctl + C_ATOM);
                ctl[C_ATOM] = 0;
                if ((unsigned long long)depth > z.maxd) z.maxd = depth;
                if (z.since_flush >= 256) {
                    z.known_total = g_add(&P.g->nodes_total, z.since_flush) + z.since_flush;
                    z.since_flush = 0;
                    if (P.inst_node_limit > 0) {
                        // the instance's own count, for its node budget
                        const unsigned long long used = g_add(&is->nodes, z.nodes) + z.nodes;
                        z.nodes = 0;
                        if (used >= (unsigned long long)P.inst_node_limit)
                            g_store_rel(&is->abandon, 1);
                    }
                }
            }
            bool descend = false;
            if (failed) {
                if (tid == 0) z.fails += 1;
            } else if (key == ~0ull) {
                // every decision variable is fixed: a solution
                if (tid == 0) {
                    z.sols += 1;
                    if (P.mode == 0) {
                        const unsigned long long idx = g_add(&is->solutions, 1ull);
                        if (P.sol_buf && (long long)idx < P.sol_cap)
                            for (int q = 0; q < ndec; ++q)
                                P.sol_buf[(size_t)idx * ndec + q] = dom(st, v.dec(q)).x;
                        g_add(&is->sol_hash, solution_hash(st, v, ndec));
                    } else {
                        const int32_t obj = dom(st, objective).x;
                        if (obj < z.local_best) z.local_best = obj;
                        const int32_t old = __hip_atomic_fetch_min(
                            &is->best, obj, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
                        if (obj < old) {
                            int32_t zz = 0;
                            while (!g_cas(&is->best_lock, zz, 1)) { zz = 0; __builtin_amdgcn_s_sleep(1); }
                            if (obj < is->pad[0]) {
                                for (int q = 0; q < ndec; ++q)
                                    P.best_vals[(size_t)inst * P.max_ndec + q] = dom(st, v.dec(q)).x;
                                is->pad[0] = obj;
                                is->best_owner = blockIdx.x;
                            }
                            g_store_rel(&is->best_lock, 0);
                        }
                    }
                }
            } else {
                descend = true;
            }
            if (descend) {
                if (depth >= P.max_depth) {
                    if (tid == 0) {
                        is->depth_overflow = 1;
                        g_store_rel(&P.g->abort, 4);
                    }
                    lds_barrier();
                    break;
                }
                if (first) {
                    // the subtree root's fixed point, kept for recomputation
                    copy_store<false, !RL>(rstb, stb, m.nI, nvars);
                    first = false;
                    if (!RL) full_barrier(); else lds_barrier();
                }
                if (LIVE) {
                    in_sel = out_sel;
                    out_sel = out_sel == 2 ? 3 : 2;
                }
                if (tid == 0) {
                    const int q = (int)(uint32_t)(key & 0xffffffffull);
                    const int x = v.dec(q);
                    const int val = dom(st, x).x;
                    // level depth; with DEP its entry also keeps where the
                    // child's trail segment starts
                    stk.put(depth, make_int4(x, val, DEP ? ctl[C_TTOP] : 0, 0));
                    if constexpr (DEP) {
                        // left child: x = lb(x), the first entry of its trail
                        Dep d1 = dp;
                        d1.trail_on = true;
                        tell_one<false>(st, d1, x, val);
                    } else {
                        tell_ub(st, x, val);  // left child: x = lb(x)
                    }
                    // donate the open right branch closest to the subtree
                    // root when other workgroups are waiting for work
                    if (P.donate && z.pf_idle > 0 && z.pf_qt - z.pf_qh < (unsigned long long)z.pf_idle) {
                        int k = -1;
                        for (int e = depth0; e <= depth; ++e)
                            if (!(stk.get(e).x & (kSideBit | kDonatedBit))) { k = e; break; }
                        if (k >= 0) {
                            const long long pp = q_claim_push(P);
                            if (pp >= 0) {
                                RecHdr *h = q_slot(P, (unsigned long long)pp);
                                int2 *dd = reinterpret_cast<int2 *>(h + 1);
                                for (int e = 0; e < k; ++e) {
                                    const int4 se = stk.get(e);
                                    dd[e] = make_int2(se.x & (0xffff | (int)kSideBit), se.y);
                                }
                                const int4 sk = stk.get(k);
                                dd[k] = make_int2((sk.x & 0xffff) | (int)kSideBit, sk.y);
                                h->inst = inst;
                                h->len = k + 1;
                                g_add(&is->outstanding, 1);
                                g_add(&P.g->outstanding, 1);
                                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
                                q_publish(P, (unsigned long long)pp);
                                stk.put(k, make_int4(sk.x | (int)kDonatedBit, sk.y, sk.z, sk.w));
                                z.don += 1;
                            }
                        }
                    }
                }
                ++depth;
                node_full = false;
                lds_barrier();
                continue;
            }
            // ---- backtrack: drop exhausted entries, flip the deepest open one
            if (tid == 0) {
                int d = depth;
                int4 sd = d > depth0 ? stk.get(d - 1) : make_int4(0, 0, 0, 0);
                while (d > depth0 && (sd.x & (kSideBit | kDonatedBit))) {
                    --d;
                    if (d > depth0) sd = stk.get(d - 1);
                }
                if (d == depth0) {
                    ctl[C_DEPTH] = -1;
                } else {
                    stk.put(d - 1, make_int4(sd.x | (int)kSideBit, sd.y, sd.z, sd.w));
                    ctl[C_DEPTH] = d;
                }
            }
            lds_barrier();
            const int nd = uni(lds_ld(&ctl[C_DEPTH]));
            if (nd < 0) {
                finished = true;
                break;
            }
            if constexpr (DEP) {
                if (nd > uni(lds_ld(ctl + C_THI))) {
                    // undo the trail of the levels below nd, deepest first
                    // (a variable changed at several levels gets the value
                    // of the shallowest), then the flipped decision
                    full_barrier();  // the trail stores of every lane are visible
                    const int top = uni(lds_ld(ctl + C_TTOP));
                    // trail segment of level k: [start kept at level k - 1,
                    // start kept at level k, or the top for the current one)
                    int e0 = uni(stk.get(depth - 1).z);
                    for (int k = depth; k >= nd; --k) {
                        const int e1 = k == depth ? top : e0;
                        if (k < depth) e0 = uni(stk.get(k - 1).z);
                        for (int i = e0 + tid; i < e1; i += W) {
                            const int4 t = gread(dp.trail + i);
                            set_dom(st, t.x, make_int2(t.y, t.z));
                        }
                        lds_barrier();
                    }
                    depth = nd;
                    if (tid == 0) {
                        const int4 dcs = stk.get(nd - 1);
                        ctl[C_TTOP] = dcs.z;
                        Dep d1 = dp;
                        d1.trail_on = true;
                        tell_one<true>(st, d1, dcs.x & 0xffff, dcs.y + 1);
                    }
                    node_full = false;
                    lds_barrier();
                    continue;
                }
                if (tid == 0) {
                    ctl[C_THI] = nd;
                    ctl[C_TTOP] = stk.get(nd - 1).z;
                }
                node_full = true;
            }
            depth = nd;
            // recompute: subtree root fixed point + decisions below it
            copy_store<!RL, false>(stb, rstb, m.nI, nvars);
            if (LIVE) {
                in_sel = 1;
                out_sel = 2;
            }
            full_barrier();  // stack levels in global memory are visible
            for (int i = depth0 + tid; i < depth; i += W) {
                const int4 e = stk.get(i);
                apply_decision(st, make_int2(e.x, e.y));
            }
            lds_barrier();
        }
        // ---- subtree done (or abandoned): publish counters
        if (tid == 0) {
            flush_counters(z, is, P.mode);
            if (finished || abandoned) {
                if (g_add(&is->outstanding, -1) == 1)
                    __hip_atomic_store(&is->t_done, (long long)wall_clock64(), __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
                g_add(&P.g->outstanding, -1);
            }
        }
        full_barrier();
    }
    if (tid == 0 && z.since_flush)
        g_add(&P.g->nodes_total, z.since_flush);
}

// One record per instance (no decisions) and the counters, before a search.
__global__ void init_search_kernel(SearchParams P)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < P.qcap) P.q_seq[i] = (i < P.ninst) ? (unsigned long long)i + 1 : (unsigned long long)i;
    if (i < P.ninst) {
        RecHdr *h = reinterpret_cast<RecHdr *>(P.q_data + (size_t)i * P.slot_bytes);
        h->inst = i;
        h->len = 0;
        InstState &s = P.inst[i];
        s.nodes = s.fails = s.solutions = s.sweeps = 0;
        s.donations = s.pops = s.sol_hash = s.max_depth = 0;
        s.ex[0] = s.ex[1] = s.ex[2] = s.ex[3] = 0;
        s.atomics = 0;
        s.t_done = 0;
        s.best = INT32_MAX;
        s.outstanding = 1;
        s.best_lock = 0;
        s.best_owner = -1;
        s.depth_overflow = 0;
        s.pad[0] = INT32_MAX;
        s.pad[1] = 0;
        s.abandon = 0;
    }
    if (i == 0) {
        SearchGlobals &g = *P.g;
        g.q_head = 0;
        g.q_tail = (unsigned long long)P.ninst;
        g.q_pushed = 0;
        g.outstanding = P.ninst;
        g.idle = 0;
        g.abort = 0;
        g.nodes_total = 0;
        g.t_start = (long long)wall_clock64();
    }
}

// ------------------------------------------------------------ MLP training
// Parameters (513 floats): W1[k][f] at k*6+f, b1 at 384+k, w2 at 448+k, b2
// at 512.  Score of a candidate: s = w2 . max(0, W1 x + b1) + b2, computed
// with one lane per hidden unit exactly as in the search (fmaf chain over
// the features, fixed-order wave sum).  Loss: mean over nodes of the
// cross-entropy between the target distribution over the node's candidates
// and the softmax of their scores.  Gradients are summed
// per wave into a partial row, then reduced in a fixed order (32 groups of
// consecutive waves in parallel, then the groups in order: deterministic),
// the last step fused with the Adam update and the bf16 copy the search
// reads.
constexpr int kPartW = 520;        // partial row: 513 gradients, loss at 513
constexpr int kMaxCand = 256;      // candidates per node in training data

__device__ inline MlpLane load_mlp_lane_f32(const float *p)
{
    MlpLane ml;
    const int k = threadIdx.x & 63;
#pragma unroll
    for (int f = 0; f < kNumFeat; ++f) ml.w1[f] = p[k * kNumFeat + f];
    ml.b1 = p[kHidden * kNumFeat + k];
    ml.w2 = p[kHidden * kNumFeat + kHidden + k];
    return ml;
}

__device__ __forceinline__ float mlp_hidden_z(const MlpLane &ml, const float *x)
{
    float z = ml.b1;
#pragma unroll
    for (int k = 0; k < kNumFeat; ++k) z = fmaf(ml.w1[k], x[k], z);
    return z;
}

__device__ __forceinline__ float wave_max_f(float x)
{
    for (int off = 32; off > 0; off >>= 1) x = fmaxf(x, __shfl_xor(x, off, 64));
    return x;
}

// one wave per node: scores, softmax, loss, dL/ds
__global__ __launch_bounds__(256) void mlp_fwd_loss_kernel(const float *params, const float *feat,
                                                           const int32_t *off, const float *target,
                                                           int nnodes, float *g, float *partial)
{
    const int lane = threadIdx.x & 63;
    const int w = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int NW = gridDim.x * (blockDim.x >> 6);
    const MlpLane ml = load_mlp_lane_f32(params);
    const float b2 = params[kNumParams - 1];
    const float invn = 1.0f / (float)nnodes;
    float loss = 0.f;
    for (int i = w; i < nnodes; i += NW) {
        const int c0 = off[i], nc = off[i + 1] - c0;
        float my[kMaxCand / 64];
#pragma unroll
        for (int r = 0; r < kMaxCand / 64; ++r) my[r] = -INFINITY;
        for (int c = 0; c < nc; ++c) {
            const float *x = feat + (size_t)(c0 + c) * kNumFeat;
            float xv[kNumFeat];
#pragma unroll
            for (int k = 0; k < kNumFeat; ++k) xv[k] = x[k];
            const float z = mlp_hidden_z(ml, xv);
            const float sc = wave_sum_f(ml.w2 * fmaxf(z, 0.f)) + b2;
#pragma unroll
            for (int r = 0; r < kMaxCand / 64; ++r)
                if (c == r * 64 + lane) my[r] = sc;
        }
        float mx = -INFINITY;
#pragma unroll
        for (int r = 0; r < kMaxCand / 64; ++r) mx = fmaxf(mx, my[r]);
        mx = wave_max_f(mx);
        float se = 0.f;
#pragma unroll
        for (int r = 0; r < kMaxCand / 64; ++r)
            se += (r * 64 + lane < nc) ? expf(my[r] - mx) : 0.f;
        se = wave_sum_f(se);
        float tv[kMaxCand / 64], ts = 0.f;
#pragma unroll
        for (int r = 0; r < kMaxCand / 64; ++r) {
            const int c = r * 64 + lane;
            tv[r] = c < nc ? target[c0 + c] : 0.f;
            ts += c < nc ? tv[r] * my[r] : 0.f;
        }
        ts = wave_sum_f(ts);
        loss += (mx + logf(se) - ts) * invn;
#pragma unroll
        for (int r = 0; r < kMaxCand / 64; ++r) {
            const int c = r * 64 + lane;
            if (c < nc)
                g[c0 + c] = (expf(my[r] - mx) / se - tv[r]) * invn;
        }
    }
    if (lane == 0) partial[(size_t)w * kPartW + kNumParams] = loss;
}

// one lane per hidden unit; waves stride over candidates
__global__ __launch_bounds__(256) void mlp_bwd_kernel(const float *params, const float *feat,
                                                      const float *g, int ncand, float *partial)
{
    const int lane = threadIdx.x & 63;
    const int w = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int NW = gridDim.x * (blockDim.x >> 6);
    const MlpLane ml = load_mlp_lane_f32(params);
    float dw1[kNumFeat] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    float db1 = 0.f, dw2 = 0.f, db2 = 0.f;
    for (int c = w; c < ncand; c += NW) {
        float xv[kNumFeat];
#pragma unroll
        for (int k = 0; k < kNumFeat; ++k) xv[k] = feat[(size_t)c * kNumFeat + k];
        const float gc = g[c];
        const float z = mlp_hidden_z(ml, xv);
        dw2 = fmaf(gc, fmaxf(z, 0.f), dw2);
        db2 += gc;
        if (z > 0.f) {
            const float dz = gc * ml.w2;
            db1 += dz;
#pragma unroll
            for (int k = 0; k < kNumFeat; ++k) dw1[k] = fmaf(dz, xv[k], dw1[k]);
        }
    }
    float *row = partial + (size_t)w * kPartW;
#pragma unroll
    for (int k = 0; k < kNumFeat; ++k) row[lane * kNumFeat + k] = dw1[k];
    row[kHidden * kNumFeat + lane] = db1;
    row[kHidden * kNumFeat + kHidden + lane] = dw2;
    if (lane == 0) row[kNumParams - 1] = db2;
}

// bf16 with round-to-nearest-even
__device__ __forceinline__ uint16_t f2bf(float x)
{
    uint32_t u = __float_as_uint(x);
    if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fc0;
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// Deterministic two-level sum of the per-wave partial rows: block (x, g)
// sums rows [g * NW / G, (g + 1) * NW / G) in order into row g of `out`;
// mlp_reduce_adam_kernel then sums the G rows in order.
constexpr int kMlpGroups = 32;
__global__ __launch_bounds__(256) void mlp_reduce_groups_kernel(const float *partial, int NW,
                                                                float *out)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p > kNumParams) return;
    const int g = blockIdx.y, w0 = g * NW / kMlpGroups, w1 = (g + 1) * NW / kMlpGroups;
    float acc = 0.f;
    for (int w = w0; w < w1; ++w) acc += partial[(size_t)w * kPartW + p];
    out[(size_t)g * kPartW + p] = acc;
}

// thread p: gradient p summed over the rows in order, then Adam
__global__ void mlp_reduce_adam_kernel(const float *partial, int NW, float *grad, float *params,
                                       float *m1, float *v1, uint16_t *wbf, float lr, int step,
                                       float *loss_out)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p > kNumParams) return;
    float acc = 0.f;
    for (int w = 0; w < NW; ++w) acc += partial[(size_t)w * kPartW + p];
    if (p == kNumParams) {
        *loss_out = acc;
        return;
    }
    grad[p] = acc;
    float x = params[p];
    if (lr > 0.f) {
        const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
        const float m = b1 * m1[p] + (1.f - b1) * acc;
        const float v = b2 * v1[p] + (1.f - b2) * acc * acc;
        m1[p] = m;
        v1[p] = v;
        const float mh = m / (1.f - powf(b1, (float)step));
        const float vh = v / (1.f - powf(b2, (float)step));
        x -= lr * mh / (sqrtf(vh) + eps);
        params[p] = x;
    }
    wbf[p] = f2bf(x);
}

__global__ void mlp_sync_bf16_kernel(const float *params, uint16_t *wbf)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < kNumParams) wbf[p] = f2bf(params[p]);
}

// scores of ncand candidates with the fp32 master or the bf16 copy
__global__ __launch_bounds__(256) void mlp_scores_kernel(const float *params, const uint16_t *wbf,
                                                         int use_bf16, const float *feat, int ncand,
                                                         float *scores)
{
    const int lane = threadIdx.x & 63;
    const int w = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int NW = gridDim.x * (blockDim.x >> 6);
    const MlpLane ml = use_bf16 ? load_mlp_lane(wbf) : load_mlp_lane_f32(params);
    const float b2 = use_bf16 ? bf16f(wbf[kNumParams - 1]) : params[kNumParams - 1];
    for (int c = w; c < ncand; c += NW) {
        float xv[kNumFeat];
#pragma unroll
        for (int k = 0; k < kNumFeat; ++k) xv[k] = feat[(size_t)c * kNumFeat + k];
        const float sc = wave_sum_f(ml.w2 * fmaxf(mlp_hidden_z(ml, xv), 0.f)) + b2;
        if (lane == 0) scores[c] = sc;
    }
}

// waves of the training launches (256 x 256 threads), then the group sums
int mlp_partial_rows() { return 256 * 4 + kMlpGroups; }

hipError_t launch_mlp_train(const float *feat, const int32_t *off, const float *target, int nnodes,
                            int ncand, float *params, float *m1, float *v1, uint16_t *wbf,
                            float *grad, float *g, float *partial, float lr, int step,
                            float *loss_dev, hipStream_t stream)
{
    const int blocks = 256;
    hipLaunchKernelGGL(mlp_fwd_loss_kernel, dim3(blocks), dim3(256), 0, stream, params, feat, off,
                       target, nnodes, g, partial);
    hipLaunchKernelGGL(mlp_bwd_kernel, dim3(blocks), dim3(256), 0, stream, params, feat, g, ncand,
                       partial);
    float *groups = partial + (size_t)blocks * 4 * kPartW;
    hipLaunchKernelGGL(mlp_reduce_groups_kernel, dim3((kNumParams + 1 + 255) / 256, kMlpGroups),
                       dim3(256), 0, stream, partial, blocks * 4, groups);
    hipLaunchKernelGGL(mlp_reduce_adam_kernel, dim3((kNumParams + 1 + 255) / 256), dim3(256), 0,
                       stream, groups, kMlpGroups, grad, params, m1, v1, wbf, lr, step, loss_dev);
    return hipGetLastError();
}

hipError_t launch_mlp_sync_bf16(const float *params, uint16_t *wbf, hipStream_t stream)
{
    hipLaunchKernelGGL(mlp_sync_bf16_kernel, dim3((kNumParams + 255) / 256), dim3(256), 0, stream,
                       params, wbf);
    return hipGetLastError();
}

hipError_t launch_mlp_scores(const float *params, const uint16_t *wbf, int use_bf16,
                             const float *feat, int ncand, float *scores, hipStream_t stream)
{
    const int blocks = ncand < 1024 ? (ncand + 3) / 4 : 256;
    hipLaunchKernelGGL(mlp_scores_kernel, dim3(blocks > 0 ? blocks : 1), dim3(256), 0, stream,
                       params, wbf, use_bf16, feat, ncand, scores);
    return hipGetLastError();
}

// ------------------------------------------------------------ launchers
size_t search_lds_bytes(size_t max_store, int max_depth, size_t max_desc, bool desc_lds, bool root_lds,
                        int feat_ndec, int list_items, size_t dep_bytes)
{
    size_t b = sizeof(int32_t) * kCtlWords + max_store;
    if (root_lds) b += max_store;
    b += align16(sizeof(int4) * (size_t)kRing);
    if (feat_ndec > 0) b += align16(32 * (size_t)feat_ndec);
    if (list_items > 0) b += 3 * align16(sizeof(uint16_t) * (size_t)list_items);
    b += dep_bytes;
    if (desc_lds) b += max_desc;
    return align16(b);
}

size_t dep_lds_bytes(int vshift, int qw, const int wcap[kDepKinds], int jcap)
{
    return align16(12 * ((size_t)1 << vshift)) + align16(4 * (size_t)qw) +
           align16(2 * (size_t)(wcap[0] + wcap[1] + wcap[2] + wcap[3] + wcap[4])) +
           align16(4 * (size_t)jcap);
}

size_t propagate_lds_bytes(size_t store, size_t desc, bool desc_lds)
{
    size_t b = sizeof(int32_t) * kCtlWords + store;
    if (desc_lds) b += desc;
    return align16(b);
}

size_t model_desc_bytes(int ndiff, int nreif, int nrows, int nterms, int ndec, int nbrows,
                        int nbslots)
{
    return desc_bytes(ndiff, nreif, nrows, nterms, ndec, nbrows, nbslots);
}

// Raise the kernel's dynamic-LDS limit where the runtime supports it; a
// launch that really does not fit still fails at launch time.
template <typename K>
static hipError_t set_lds_limit(K kernel, size_t bytes)
{
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(kernel),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    (void)hipGetLastError();
    return hipSuccess;
}

hipError_t launch_propagate_batch(const DevModel *m_dev, int nbox, const int32_t *lb_in,
                                  const int32_t *ub_in, int32_t *lb_out, int32_t *ub_out,
                                  int32_t *status, int32_t *sweeps, int grid, int block,
                                  size_t lds, bool desc_lds, hipStream_t stream)
{
    if (desc_lds) {
        hipError_t e = set_lds_limit(propagate_batch_kernel<true>, lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(propagate_batch_kernel<true>, dim3(grid), dim3(block), lds, stream,
                           m_dev, nbox, lb_in, ub_in, lb_out, ub_out, status, sweeps);
    } else {
        hipError_t e = set_lds_limit(propagate_batch_kernel<false>, lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(propagate_batch_kernel<false>, dim3(grid), dim3(block), lds, stream,
                           m_dev, nbox, lb_in, ub_in, lb_out, ub_out, status, sweeps);
    }
    return hipGetLastError();
}

hipError_t launch_propagate_incr(const DevModel *m_dev, const IncrParams &A, int grid, int block,
                                 size_t lds, hipStream_t stream)
{
    hipError_t e = set_lds_limit(propagate_incr_kernel, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(propagate_incr_kernel, dim3(grid), dim3(block), lds, stream, m_dev, A);
    return hipGetLastError();
}

// the search kernel variant for a layout, branching rule, propagation mode
// (0 every propagator every sweep, 1 item lists, 2 dependency-driven) and
// occupancy class
template <bool L, int PM, bool H>
static const void *search_fn_lv(bool desc_lds, bool root_lds)
{
    if (desc_lds && root_lds) return reinterpret_cast<const void *>(search_kernel<true, true, L, PM, H>);
    if (desc_lds) return reinterpret_cast<const void *>(search_kernel<true, false, L, PM, H>);
    if (root_lds) return reinterpret_cast<const void *>(search_kernel<false, true, L, PM, H>);
    return reinterpret_cast<const void *>(search_kernel<false, false, L, PM, H>);
}

template <bool L, bool H>
static const void *search_fn_l(const SearchShape &k)
{
    if (k.dep) return search_fn_lv<L, 2, H>(k.desc_lds, k.root_lds);
    if (k.live) return search_fn_lv<L, 1, H>(k.desc_lds, k.root_lds);
    return search_fn_lv<L, 0, H>(k.desc_lds, k.root_lds);
}

template <bool H>
static const void *search_fn_h(const SearchShape &k)
{
    return k.learned ? search_fn_l<true, H>(k) : search_fn_l<false, H>(k);
}

static const void *search_fn(const SearchShape &k)
{
    return k.hi ? search_fn_h<true>(k) : search_fn_h<false>(k);
}

hipError_t launch_search(const SearchParams &P, int grid, int block, size_t lds,
                         const SearchShape &k, hipStream_t stream)
{
    const int n = P.qcap > P.ninst ? P.qcap : P.ninst;
    hipLaunchKernelGGL(init_search_kernel, dim3((n + 255) / 256), dim3(256), 0, stream, P);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const void *fn = search_fn(k);
    e = set_lds_limit(fn, lds);
    if (e != hipSuccess) return e;
    SearchParams p = P;
    void *args[] = {&p};
    e = hipLaunchKernel(fn, dim3(grid), dim3(block), args, lds, stream);
    if (e != hipSuccess) return e;
    return hipGetLastError();
}

// The same two launches as one hipGraph (two kernel nodes, the search
// depending on the initialisation; no memset nodes).
hipError_t build_search_graph(const SearchParams &P, int grid, int block, size_t lds,
                              const SearchShape &k, hipGraphExec_t *exec)
{
    const void *fn = search_fn(k);
    hipError_t e = set_lds_limit(fn, lds);
    if (e != hipSuccess) return e;
    hipGraph_t g = nullptr;
    if ((e = hipGraphCreate(&g, 0)) != hipSuccess) return e;
    SearchParams p = P;
    void *args[] = {&p};
    const int n = P.qcap > P.ninst ? P.qcap : P.ninst;
    hipKernelNodeParams kp{};
    kp.func = reinterpret_cast<void *>(init_search_kernel);
    kp.gridDim = dim3((n + 255) / 256);
    kp.blockDim = dim3(256);
    kp.sharedMemBytes = 0;
    kp.kernelParams = args;
    kp.extra = nullptr;
    hipGraphNode_t n_init = nullptr, n_search = nullptr;
    e = hipGraphAddKernelNode(&n_init, g, nullptr, 0, &kp);
    if (e == hipSuccess) {
        hipKernelNodeParams ks = kp;
        ks.func = const_cast<void *>(fn);
        ks.gridDim = dim3(grid);
        ks.blockDim = dim3(block);
        ks.sharedMemBytes = (unsigned)lds;
        e = hipGraphAddKernelNode(&n_search, g, &n_init, 1, &ks);
    }
    if (e == hipSuccess) e = hipGraphInstantiate(exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    return e;
}

// The workspace of the search entry point that allocates nothing (for
// callers that cannot call hipMalloc).  Every device the library is loaded
// on holds one copy until the process ends; in host code the name stands
// for no device address, so kernels get the address that
// hipGetSymbolAddress returns on the device that runs them.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

hipError_t scratch_address(void **ptr)
{
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static void *addr[kMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        addr[dev] = p;
    }
    *ptr = addr[dev];
    return hipSuccess;
}

hipError_t search_occupancy(int block, size_t lds, const SearchShape &k, int *wgs_per_cu)
{
    const void *fn = search_fn(k);
    hipError_t e = set_lds_limit(fn, lds);
    if (e != hipSuccess) return e;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(wgs_per_cu, fn, block, lds);
}

}  // namespace pccp
