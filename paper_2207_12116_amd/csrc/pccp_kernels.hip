// HIP kernels of libpccp for gfx950 (CDNA4): lock-free parallel propagation
// to a fixed point over int32 interval stores, and depth-first
// propagate-and-search over a device-side queue of subtrees.
//
// Design (the paper's own GPU solver, §5, was written for a Turing laptop
// GPU; this keeps what holds on gfx950 and changes the rest):
//   * One workgroup per subproblem (§5: one block per subproblem).  The
//     store of the subproblem (lb[], ub[] as int32 SoA) lives in LDS.
//   * Every propagator runs every sweep (eventless propagation, §5).  Each
//     lane takes descriptors t = tid, tid + W, ... of each kind in turn
//     (§5, fixed point loop: strided loop over the propagators).
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
//     three rotating LDS words; one barrier per sweep (§5, has_changed[3]).
//     The barrier is an LDS-only fence + s_barrier, so global loads issued
//     by the control lane stay in flight across sweeps.
//   * Failure (an empty interval, §5) is flagged in-loop whenever a tell
//     crosses the opposite bound it read, which bounds the number of sweeps
//     on failing stores, and confirmed by a scan of the store at the fixed
//     point (§5: failure can be examined after the loop).
//   * Search (§5): full recomputation on backtracking.  Each workgroup keeps
//     the fixed point of its subproblem's root; a backtrack copies it back
//     and re-applies the decisions of the new path.  Descending keeps the
//     current store.  Embarrassingly parallel search with dynamically
//     generated subproblems (§5): a workgroup donates the right branch
//     closest to its subproblem root to a bounded lock-free MPMC queue when
//     other workgroups are idle.
//
// No MFMA: the work is integer lattice arithmetic, bound by LDS traffic and
// barrier latency.
#include <hip/hip_runtime.h>
#include <stdint.h>

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
__device__ __forceinline__ uint32_t gread(const uint32_t *p) { return (uint32_t) * (g_i32 *)p; }
__device__ __forceinline__ void gwrite(int32_t *p, int32_t v) { *(g_i32w *)p = v; }

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
};

// ------------------------------------------------------------ descriptors
// Descriptor tables of one instance, in LDS (DL) or in global memory.
template <bool DL>
struct View {
    int32_t nvars, ndiff, nreif, nrows, ndec, objective;
    const int2 *diff_;
    const int2 *reif_;
    const int4 *rows_;
    const uint32_t *terms_;
    const int32_t *dec_;
    __device__ __forceinline__ int2 diff(int t) const { return DL ? diff_[t] : gread(diff_ + t); }
    __device__ __forceinline__ int2 reif(int t) const { return DL ? reif_[t] : gread(reif_ + t); }
    __device__ __forceinline__ int4 rows(int t) const { return DL ? rows_[t] : gread(rows_ + t); }
    __device__ __forceinline__ uint32_t terms(int t) const { return DL ? terms_[t] : gread(terms_ + t); }
    __device__ __forceinline__ int32_t dec(int t) const { return DL ? dec_[t] : gread(dec_ + t); }
};

__host__ __device__ inline size_t align16(size_t x) { return (x + 15) & ~size_t(15); }

__host__ __device__ inline size_t desc_bytes(int ndiff, int nreif, int nrows, int nterms, int ndec)
{
    return align16(sizeof(int4) * (size_t)nrows) + align16(sizeof(int2) * (size_t)ndiff) +
           align16(sizeof(int2) * (size_t)nreif) + align16(sizeof(uint32_t) * (size_t)nterms) +
           align16(sizeof(int32_t) * (size_t)ndec);
}

// View over global memory.
__device__ inline View<false> view_global(const DevModel &m)
{
    View<false> v;
    v.nvars = m.nvars; v.ndiff = m.ndiff; v.nreif = m.nreif; v.nrows = m.nrows;
    v.ndec = m.ndec; v.objective = m.objective;
    v.diff_ = m.diff; v.reif_ = m.reif; v.rows_ = m.rows; v.terms_ = m.terms; v.dec_ = m.dec;
    return v;
}

// Copy the descriptor tables into LDS at `dst` (all threads) and return a
// view over the copy.  Caller puts a barrier before the view is used.
__device__ inline View<true> stage_descriptors(const DevModel &m, char *dst)
{
    const int tid = threadIdx.x, W = blockDim.x;
    View<true> v;
    v.nvars = m.nvars; v.ndiff = m.ndiff; v.nreif = m.nreif; v.nrows = m.nrows;
    v.ndec = m.ndec; v.objective = m.objective;
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
    for (int i = tid; i < m.nrows; i += W) rows[i] = gread(m.rows + i);
    for (int i = tid; i < m.ndiff; i += W) diff[i] = gread(m.diff + i);
    for (int i = tid; i < m.nreif; i += W) reif[i] = gread(m.reif + i);
    for (int i = tid; i < m.nterms; i += W) terms[i] = gread(m.terms + i);
    for (int i = tid; i < m.ndec; i += W) dec[i] = gread(m.dec + i);
    v.rows_ = rows; v.diff_ = diff; v.reif_ = reif; v.terms_ = terms; v.dec_ = dec;
    return v;
}

// ------------------------------------------------------ propagation loop
// Fixed point of the LDS store (lb, ub) under every propagator of `v`.
// Returns 1 if the loop saw a failure, 0 at a fixed point (the post scan
// still has to look for an empty interval the loop did not see).
// Precondition: a barrier separates this call from any earlier read of the
// control words C_FLAG*, C_POSTFAIL, C_KEY.
template <bool DL>
__device__ int propagate_wg(const View<DL> &v, int32_t *lb, int32_t *ub, int32_t *ctl,
                            uint32_t &nsweeps)
{
    const int tid = threadIdx.x, W = blockDim.x;
    const int lane = tid & 63;
    if (tid == 0) {
        ctl[C_FLAG0] = 0;
        ctl[C_FLAG1] = 0;
        ctl[C_FLAG2] = 0;
        ctl[C_POSTFAIL] = 0;
        *reinterpret_cast<unsigned long long *>(ctl + C_KEY) = ~0ull;
    }
    lds_barrier();
    int slot = 0;
    for (;;) {
        bool chg = false, bad = false;
        // kind 1: x - y <= c  =>  ub(x) <= c + ub(y),  lb(y) >= lb(x) - c
        for (int t = tid; t < v.ndiff; t += W) {
            const int2 e = v.diff(t);
            const int x = e.x & 0xffff, y = (uint32_t)e.x >> 16;
            const int c = e.y;
            const int lbx = lds_ld(&lb[x]), ubx = lds_ld(&ub[x]);
            const int lby = lds_ld(&lb[y]), uby = lds_ld(&ub[y]);
            const int u = c + uby;
            if (u < ubx) { join_ub(&ub[x], u); chg = true; bad |= u < lbx; }
            const int l = lbx - c;
            if (l > lby) { join_lb(&lb[y], l); chg = true; bad |= l > uby; }
        }
        // kind 2: b <=> (si <= sj and sj < si + d), the four guarded
        // processes of [[phi <=> psi]] with interval entailment
        for (int t = tid; t < v.nreif; t += W) {
            const int2 e = v.reif(t);
            const int b = e.x & 0xffff, i = (uint32_t)e.x >> 16;
            const int j = e.y & 0xffff, d = e.y >> 16;
            const int lbi = lds_ld(&lb[i]), ubi = lds_ld(&ub[i]);
            const int lbj = lds_ld(&lb[j]), ubj = lds_ld(&ub[j]);
            const int lbb = lds_ld(&lb[b]), ubb = lds_ld(&ub[b]);
            const bool E1 = ubi <= lbj;              // entailed(si <= sj)
            const bool E2 = ubj <= lbi + d - 1;      // entailed(sj < si + d)
            if (lbb < 1 && E1 && E2) { join_lb(&lb[b], 1); chg = true; bad |= ubb < 1; }
            if (ubb > 0 && (lbi > ubj || lbj >= ubi + d)) {
                join_ub(&ub[b], 0); chg = true; bad |= lbb > 0;
            }
            if (lbb >= 1) {                          // b  =>  si <= sj <= si + d - 1
                if (ubj < ubi) { join_ub(&ub[i], ubj); chg = true; bad |= ubj < lbi; }
                if (lbi > lbj) { join_lb(&lb[j], lbi); chg = true; bad |= lbi > ubj; }
                const int u = ubi + d - 1;
                if (u < ubj) { join_ub(&ub[j], u); chg = true; bad |= u < lbj; }
                const int l = lbj - d + 1;
                if (l > lbi) { join_lb(&lb[i], l); chg = true; bad |= l > ubi; }
            }
            if (ubb <= 0) {                          // not b  =>  sj < si  or  sj >= si + d
                if (E1) {
                    const int l = lbi + d;
                    if (l > lbj) { join_lb(&lb[j], l); chg = true; bad |= l > ubj; }
                    const int u = ubj - d;
                    if (u < ubi) { join_ub(&ub[i], u); chg = true; bad |= u < lbi; }
                }
                if (E2) {
                    const int u = ubi - 1;
                    if (u < ubj) { join_ub(&ub[j], u); chg = true; bad |= u < lbj; }
                    const int l = lbj + 1;
                    if (l > lbi) { join_lb(&lb[i], l); chg = true; bad |= l > ubi; }
                }
            }
        }
        // kind 3: sum_t a_t x_t <= rhs.  S = sum of each term's smallest
        // value; the tell on x_t is a_t x_t <= rhs - (S - m_t).  A term
        // re-read after S was formed can only have grown, which makes the
        // tell weaker, never unsound; the final change-free sweep reads a
        // constant store and is exact.
        for (int r = tid; r < v.nrows; r += W) {
            const int4 rd = v.rows(r);
            const int t0 = rd.x, t1 = rd.x + rd.y, rhs = rd.z;
            int S = 0;
            for (int t = t0; t < t1; ++t) {
                const uint32_t tv = v.terms(t);
                const int x = tv & 0xffff, a = (int32_t)tv >> 16;
                S += a > 0 ? a * lds_ld(&lb[x]) : a * lds_ld(&ub[x]);
            }
            for (int t = t0; t < t1; ++t) {
                const uint32_t tv = v.terms(t);
                const int x = tv & 0xffff, a = (int32_t)tv >> 16;
                if (a > 0) {
                    const int lbx = lds_ld(&lb[x]), ubx = lds_ld(&ub[x]);
                    const int rr = rhs - (S - a * lbx);      // a x <= rr
                    if (rr < a * ubx) {
                        const int nb = a == 1 ? rr : floor_div_pos(rr, a);
                        join_ub(&ub[x], nb); chg = true; bad |= nb < lbx;
                    }
                } else {
                    const int lbx = lds_ld(&lb[x]), ubx = lds_ld(&ub[x]);
                    const int rr = rhs - (S - a * ubx);      // a x <= rr, a < 0
                    if (rr < a * lbx) {                      // x >= ceil(rr / a)
                        const int nb = a == -1 ? -rr : -floor_div_pos(rr, -a);
                        join_lb(&lb[x], nb); chg = true; bad |= nb > ubx;
                    }
                }
            }
        }
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
    }
}

// After the loop: look for an empty interval anywhere in the store and, if
// `branch` is set, find the branching variable (smallest key among unfixed
// decision variables).  Ends with a barrier; results in ctl[C_POSTFAIL] and
// the 64-bit word at ctl[C_KEY] (~0 when every decision variable is fixed).
template <bool DL>
__device__ void post_scan(const View<DL> &v, const int32_t *lb, const int32_t *ub, int32_t *ctl,
                          int branching, bool branch)
{
    const int tid = threadIdx.x, W = blockDim.x, lane = tid & 63;
    bool bad = false;
    for (int x = tid; x < v.nvars; x += W)
        bad |= lds_ld(&lb[x]) > lds_ld(&ub[x]);
    unsigned long long key = ~0ull;
    if (branch) {
        for (int q = tid; q < v.ndec; q += W) {
            const int x = v.dec(q);
            const int w = lds_ld(&ub[x]) - lds_ld(&lb[x]);
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
    const int tid = threadIdx.x, W = blockDim.x;
    int32_t *ctl = reinterpret_cast<int32_t *>(smem);
    int32_t *lb = ctl + kCtlWords;
    int32_t *ub = lb + ((m.nvars + 3) & ~3);
    char *dsc = reinterpret_cast<char *>(ub + ((m.nvars + 3) & ~3));
    View<DL> v;
    if constexpr (DL) v = stage_descriptors(m, dsc); else v = view_global(m);
    for (int box = blockIdx.x; box < nbox; box += gridDim.x) {
        const size_t off = (size_t)box * m.nvars;
        for (int x = tid; x < m.nvars; x += W) {
            lb[x] = gread(lb_in + off + x);
            ub[x] = gread(ub_in + off + x);
        }
        uint32_t nsw = 0;
        lds_barrier();
        const int st = propagate_wg(v, lb, ub, ctl, nsw);
        post_scan(v, lb, ub, ctl, 0, false);
        const int failed = st | lds_ld(&ctl[C_POSTFAIL]);
        for (int x = tid; x < m.nvars; x += W) {
            gwrite(lb_out + off + x, lb[x]);
            gwrite(ub_out + off + x, ub[x]);
        }
        if (tid == 0) {
            status[box] = failed;
            if (sweeps) sweeps[box] = (int32_t)nsw;
        }
        lds_barrier();
    }
}

// ------------------------------------------------------------ the queue
// Bounded lock-free MPMC queue of subtree records (D. Vyukov's bounded
// queue: one sequence number per slot).  Only lane 0 of a workgroup calls
// these.
__device__ long long q_claim_pop(const SearchParams &P)
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

__device__ void q_release_slot(const SearchParams &P, unsigned long long pos)
{
    g_store_rel(&P.q_seq[pos % (unsigned)P.qcap], pos + (unsigned long long)P.qcap);
}

__device__ long long q_claim_push(const SearchParams &P)
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

__device__ void q_publish(const SearchParams &P, unsigned long long pos)
{
    g_store_rel(&P.q_seq[pos % (unsigned)P.qcap], pos + 1);
}

__device__ inline RecHdr *q_slot(const SearchParams &P, unsigned long long pos)
{
    return reinterpret_cast<RecHdr *>(P.q_data + (size_t)(pos % (unsigned)P.qcap) * P.slot_bytes);
}

// FNV-1a 64 over the little-endian bytes, finalised by MurmurHash3 fmix64.
template <bool DL>
__device__ unsigned long long solution_hash(const int32_t *lb, const View<DL> &v, int n)
{
    unsigned long long h = 0xcbf29ce484222325ull;
    for (int i = 0; i < n; ++i) {
        const uint32_t val = (uint32_t)lb[v.dec(i)];
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

// apply decision word (var | side << 16, val) to the store as a join
__device__ __forceinline__ void apply_decision(int32_t *lb, int32_t *ub, int2 dcs)
{
    const int x = dcs.x & 0xffff;
    if (dcs.x & kSideBit)
        join_lb(&lb[x], dcs.y + 1);
    else
        join_ub(&ub[x], dcs.y);
}

// ------------------------------------------------------------ search
// Persistent kernel: every workgroup loops { take a subtree record; DFS it }
// until the queue is empty and no subtree is in progress, or a limit hits.
template <bool DL, bool RL>
__global__ __launch_bounds__(1024) void search_kernel(SearchParams P)
{
    extern __shared__ __align__(16) char smem[];
    const int tid = threadIdx.x, W = blockDim.x;
    const int Vp = (P.max_vars + 3) & ~3;
    int32_t *ctl = reinterpret_cast<int32_t *>(smem);
    int32_t *lb = ctl + kCtlWords;
    int32_t *ub = lb + Vp;
    int32_t *rlb, *rub;
    char *after;
    if (RL) {
        rlb = ub + Vp;
        rub = rlb + Vp;
        after = reinterpret_cast<char *>(rub + Vp);
    } else {
        rlb = P.root_scratch + (size_t)blockIdx.x * 2 * Vp;
        rub = rlb + Vp;
        after = reinterpret_cast<char *>(ub + Vp);
    }
    int2 *stack = reinterpret_cast<int2 *>(after);
    char *dsc = reinterpret_cast<char *>(after) + align16(sizeof(int2) * (size_t)P.max_depth);

    // lane-0 private counters
    unsigned long long c_nodes = 0, c_fails = 0, c_sols = 0, c_sweeps = 0, c_don = 0;
    unsigned long long c_maxd = 0;
    unsigned long long since_flush = 0, known_total = 0;
    int32_t local_best = INT32_MAX;
    // lane-0 copies of global words, loaded during one node and used at the
    // next, so that their latency overlaps the propagation
    int32_t pf_best = INT32_MAX, pf_abort = 0, pf_idle = 0;
    unsigned long long pf_qt = 0, pf_qh = 0;
    long long t_start = 0;
    if (tid == 0) t_start = g_load(&P.g->t_start);
    int cur_inst = -1;
    View<DL> v{};
    DevModel m{};
    bool idle_reg = false;

    for (;;) {
        // ---- take a record (lane 0)
        if (tid == 0) {
            long long got = -2;
            for (;;) {
                if (g_load(&P.g->abort) != 0) { got = -2; break; }
                const long long pos = q_claim_pop(P);
                if (pos >= 0) { got = pos; break; }
                if (g_load_acq(&P.g->outstanding) == 0) { got = -2; break; }
                if (P.t_limit_ticks > 0 && (long long)wall_clock64() - t_start > P.t_limit_ticks) {
                    g_store_rel(&P.g->abort, 2);
                    got = -2;
                    break;
                }
                if (!idle_reg) { g_add(&P.g->idle, 1); idle_reg = true; }
                __builtin_amdgcn_s_sleep(8);
            }
            if (got >= 0 && idle_reg) { g_add(&P.g->idle, -1); idle_reg = false; }
            ctl[C_SLOT] = (int32_t)(got & 0xffffffff);
            ctl[C_SLOT_HI] = (int32_t)(got >> 32);
            if (got >= 0) {
                const RecHdr *h = q_slot(P, (unsigned long long)got);
                ctl[C_INST] = h->inst;
                ctl[C_LEN] = h->len;
            }
        }
        full_barrier();
        const long long pos = (long long)(((unsigned long long)(uint32_t)ctl[C_SLOT_HI] << 32) |
                                          (uint32_t)ctl[C_SLOT]);
        if (pos < 0)
            break;
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        const int inst = ctl[C_INST];
        const int len = ctl[C_LEN];
        const int2 *rec = reinterpret_cast<const int2 *>(q_slot(P, (unsigned long long)pos) + 1);
        for (int i = tid; i < len; i += W) {
            const int2 dcs = rec[i];
            stack[i] = make_int2(dcs.x & (0xffff | (int)kSideBit), dcs.y);
        }
        if (inst != cur_inst) {
            if (tid == 0) local_best = INT32_MAX;
            m = P.models[inst];
            if constexpr (DL) v = stage_descriptors(m, dsc); else v = view_global(m);
            cur_inst = inst;
        }
        for (int x = tid; x < m.nvars; x += W) {
            lb[x] = gread(m.lb0 + x);
            ub[x] = gread(m.ub0 + x);
        }
        lds_barrier();
        for (int i = tid; i < len; i += W)
            apply_decision(lb, ub, stack[i]);
        full_barrier();  // every lane is done reading the record
        if (tid == 0)
            q_release_slot(P, (unsigned long long)pos);

        const int depth0 = len;
        int depth = len;
        bool first = true;
        bool finished = false;
        InstState *is = &P.inst[inst];
        if (tid == 0) {
            pf_best = g_load(&is->best);
            pf_abort = 0;
        }
        // ---- depth-first search of this subtree
        for (;;) {
            if (tid == 0) {
                int stop = pf_abort != 0;
                if (P.node_limit > 0 && known_total + since_flush >= (unsigned long long)P.node_limit) {
                    g_store_rel(&P.g->abort, 1);
                    stop = 1;
                }
                if (P.t_limit_ticks > 0 && (long long)wall_clock64() - t_start > P.t_limit_ticks) {
                    g_store_rel(&P.g->abort, 2);
                    stop = 1;
                }
                if (P.cancel && (c_nodes & 255) == 0 && *P.cancel != 0) {
                    g_store_rel(&P.g->abort, 3);
                    stop = 1;
                }
                ctl[C_STOP] = stop;
                if (!stop && P.mode == 1) {
                    local_best = pf_best < local_best ? pf_best : local_best;
                    if (local_best != INT32_MAX)
                        join_ub(&ub[m.objective], local_best - 1);
                }
                pf_best = g_load(&is->best);
                pf_abort = g_load(&P.g->abort);
                if (P.donate) {
                    pf_idle = g_load(&P.g->idle);
                    pf_qt = g_load(&P.g->q_tail);
                    pf_qh = g_load(&P.g->q_head);
                }
            }
            lds_barrier();
            if (lds_ld(&ctl[C_STOP]))
                break;
            uint32_t nsw = 0;
            const int st = propagate_wg(v, lb, ub, ctl, nsw);
            post_scan(v, lb, ub, ctl, P.branching, st == 0);
            const int failed = st | lds_ld(&ctl[C_POSTFAIL]);
            const unsigned long long key =
                *reinterpret_cast<volatile unsigned long long *>(ctl + C_KEY);
            if (tid == 0) {
                ++c_nodes;
                ++since_flush;
                c_sweeps += nsw;
                if ((unsigned long long)depth > c_maxd) c_maxd = depth;
                if (since_flush >= 256) {
                    known_total = g_add(&P.g->nodes_total, since_flush) + since_flush;
                    since_flush = 0;
                }
            }
            bool descend = false;
            if (failed) {
                if (tid == 0) ++c_fails;
            } else if (key == ~0ull) {
                // every decision variable is fixed: a solution
                if (tid == 0) {
                    ++c_sols;
                    if (P.mode == 0) {
                        const unsigned long long idx = g_add(&is->solutions, 1ull);
                        if (P.sol_buf && (long long)idx < P.sol_cap)
                            for (int q = 0; q < m.ndec; ++q)
                                P.sol_buf[(size_t)idx * m.ndec + q] = lb[v.dec(q)];
                        g_add(&is->sol_hash, solution_hash(lb, v, m.ndec));
                    } else {
                        const int32_t obj = lb[m.objective];
                        local_best = obj < local_best ? obj : local_best;
                        const int32_t old = __hip_atomic_fetch_min(
                            &is->best, obj, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
                        if (obj < old) {
                            int32_t z = 0;
                            while (!g_cas(&is->best_lock, z, 1)) { z = 0; __builtin_amdgcn_s_sleep(1); }
                            if (obj < is->pad[0]) {
                                for (int q = 0; q < m.ndec; ++q)
                                    P.best_vals[(size_t)inst * P.max_ndec + q] = lb[v.dec(q)];
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
                    for (int x = tid; x < m.nvars; x += W) {
                        if (RL) {
                            rlb[x] = lb[x];
                            rub[x] = ub[x];
                        } else {
                            gwrite(rlb + x, lb[x]);
                            gwrite(rub + x, ub[x]);
                        }
                    }
                    first = false;
                    if (!RL) full_barrier(); else lds_barrier();
                }
                if (tid == 0) {
                    const int q = (int)(uint32_t)(key & 0xffffffffull);
                    const int x = v.dec(q);
                    const int val = lb[x];
                    stack[depth] = make_int2(x, val);
                    ub[x] = val;  // left child: x = lb(x)
                    // donate the open right branch closest to the subtree
                    // root when other workgroups are waiting for work
                    if (P.donate) {
                        const int idle = pf_idle;
                        if (idle > 0) {
                            const unsigned long long qs = pf_qt - pf_qh;
                            if (qs < (unsigned long long)idle) {
                                int k = -1;
                                for (int e = depth0; e <= depth; ++e)
                                    if (!(stack[e].x & (kSideBit | kDonatedBit))) { k = e; break; }
                                if (k >= 0) {
                                    const long long pp = q_claim_push(P);
                                    if (pp >= 0) {
                                        RecHdr *h = q_slot(P, (unsigned long long)pp);
                                        int2 *dd = reinterpret_cast<int2 *>(h + 1);
                                        for (int e = 0; e < k; ++e)
                                            dd[e] = make_int2(stack[e].x & (0xffff | (int)kSideBit), stack[e].y);
                                        dd[k] = make_int2((stack[k].x & 0xffff) | (int)kSideBit, stack[k].y);
                                        h->inst = inst;
                                        h->len = k + 1;
                                        g_add(&is->outstanding, 1);
                                        g_add(&P.g->outstanding, 1);
                                        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
                                        q_publish(P, (unsigned long long)pp);
                                        stack[k].x |= (int)kDonatedBit;
                                        ++c_don;
                                    }
                                }
                            }
                        }
                    }
                }
                ++depth;
                lds_barrier();
                continue;
            }
            // ---- backtrack: drop exhausted entries, flip the deepest open one
            if (tid == 0) {
                int d = depth;
                while (d > depth0 && (stack[d - 1].x & (kSideBit | kDonatedBit))) --d;
                if (d == depth0) {
                    ctl[C_DEPTH] = -1;
                } else {
                    stack[d - 1].x |= (int)kSideBit;
                    ctl[C_DEPTH] = d;
                }
            }
            lds_barrier();
            const int nd = lds_ld(&ctl[C_DEPTH]);
            if (nd < 0) {
                finished = true;
                break;
            }
            depth = nd;
            // recompute: subtree root fixed point + decisions below it
            for (int x = tid; x < m.nvars; x += W) {
                lb[x] = RL ? rlb[x] : gread(rlb + x);
                ub[x] = RL ? rub[x] : gread(rub + x);
            }
            lds_barrier();
            for (int i = depth0 + tid; i < depth; i += W)
                apply_decision(lb, ub, stack[i]);
            lds_barrier();
        }
        // ---- subtree done (or abandoned): publish counters
        if (tid == 0) {
            g_add(&is->nodes, c_nodes);
            g_add(&is->fails, c_fails);
            g_add(&is->sweeps, c_sweeps);
            g_add(&is->donations, c_don);
            g_add(&is->pops, 1ull);
            if (P.mode == 1) g_add(&is->solutions, c_sols);
            __hip_atomic_fetch_max(&is->max_depth, c_maxd, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            c_nodes = c_fails = c_sweeps = c_don = c_sols = c_maxd = 0;
            if (finished) {
                if (g_add(&is->outstanding, -1) == 1)
                    __hip_atomic_store(&is->t_done, (long long)wall_clock64(), __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
                g_add(&P.g->outstanding, -1);
            }
        }
        full_barrier();
    }
    if (tid == 0 && since_flush)
        g_add(&P.g->nodes_total, since_flush);
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
        s.t_done = 0;
        s.best = INT32_MAX;
        s.outstanding = 1;
        s.best_lock = 0;
        s.best_owner = -1;
        s.depth_overflow = 0;
        s.pad[0] = INT32_MAX;
        s.pad[1] = s.pad[2] = 0;
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

// ------------------------------------------------------------ launchers
size_t search_lds_bytes(int max_vars, int max_depth, size_t max_desc, bool desc_lds, bool root_lds)
{
    const size_t Vp = (size_t)((max_vars + 3) & ~3);
    size_t b = sizeof(int32_t) * kCtlWords + 2 * Vp * sizeof(int32_t);
    if (root_lds) b += 2 * Vp * sizeof(int32_t);
    b += align16(sizeof(int2) * (size_t)max_depth);
    if (desc_lds) b += max_desc;
    return align16(b);
}

size_t propagate_lds_bytes(int nvars, size_t desc, bool desc_lds)
{
    const size_t Vp = (size_t)((nvars + 3) & ~3);
    size_t b = sizeof(int32_t) * kCtlWords + 2 * Vp * sizeof(int32_t);
    if (desc_lds) b += desc;
    return align16(b);
}

size_t model_desc_bytes(int ndiff, int nreif, int nrows, int nterms, int ndec)
{
    return desc_bytes(ndiff, nreif, nrows, nterms, ndec);
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

hipError_t launch_search(const SearchParams &P, int grid, int block, size_t lds, bool desc_lds,
                         bool root_lds, hipStream_t stream)
{
    const int n = P.qcap > P.ninst ? P.qcap : P.ninst;
    hipLaunchKernelGGL(init_search_kernel, dim3((n + 255) / 256), dim3(256), 0, stream, P);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
#define PCCP_LAUNCH(DLV, RLV)                                                                  \
    do {                                                                                       \
        e = set_lds_limit(search_kernel<DLV, RLV>, lds);                                       \
        if (e != hipSuccess) return e;                                                         \
        hipLaunchKernelGGL((search_kernel<DLV, RLV>), dim3(grid), dim3(block), lds, stream, P); \
    } while (0)
    if (desc_lds && root_lds) PCCP_LAUNCH(true, true);
    else if (desc_lds) PCCP_LAUNCH(true, false);
    else if (root_lds) PCCP_LAUNCH(false, true);
    else PCCP_LAUNCH(false, false);
#undef PCCP_LAUNCH
    return hipGetLastError();
}

hipError_t search_occupancy(int block, size_t lds, bool desc_lds, bool root_lds, int *wgs_per_cu)
{
    hipError_t e;
#define PCCP_OCC(DLV, RLV)                                                                     \
    do {                                                                                       \
        e = set_lds_limit(search_kernel<DLV, RLV>, lds);                                       \
        if (e != hipSuccess) return e;                                                         \
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(wgs_per_cu, search_kernel<DLV, RLV>,  \
                                                         block, lds);                          \
    } while (0)
    if (desc_lds && root_lds) PCCP_OCC(true, true);
    else if (desc_lds) PCCP_OCC(true, false);
    else if (root_lds) PCCP_OCC(false, true);
    else PCCP_OCC(false, false);
#undef PCCP_OCC
    return e;
}

}  // namespace pccp
