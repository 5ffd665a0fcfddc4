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
};

// ------------------------------------------------------------ descriptors
// Descriptor tables of one instance, in LDS (DL) or in global memory.
template <bool DL>
struct View {
    int32_t nvars, ndiff, nreif, nrows, ndec, objective;
    int32_t row_group, row_chunks;
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
    // learned-branching tables (always in global memory)
    const float *fstat;
    const int32_t *fr_ptr;
    const int2 *fr;
    const int32_t *fb_ptr;
    const int32_t *fb;
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
    v.row_group = m.row_group; v.row_chunks = m.row_chunks;
    v.diff_ = m.diff; v.reif_ = m.reif; v.rows_ = m.rows; v.terms_ = m.terms; v.dec_ = m.dec;
    v.fstat = m.fstat; v.fr_ptr = m.fr_ptr; v.fr = m.fr; v.fb_ptr = m.fb_ptr; v.fb = m.fb;
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
    v.row_group = m.row_group; v.row_chunks = m.row_chunks;
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
    v.fstat = m.fstat; v.fr_ptr = m.fr_ptr; v.fr = m.fr; v.fb_ptr = m.fb_ptr; v.fb = m.fb;
    return v;
}

// ------------------------------------------------------ propagation loop
// Each lane issues the loads of several propagators before it uses any of
// them (U items per chunk), so one sweep costs a few LDS round trips per
// chunk rather than two per propagator.  Indices past the end of a table are
// clamped to its last entry and the item is masked out of the tells.

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

// kind 1: x - y <= c  =>  ub(x) <= c + ub(y),  lb(y) >= lb(x) - c
template <bool DL>
__device__ __forceinline__ void sweep_diff(const View<DL> &v, int32_t *lb, int32_t *ub,
                                           bool &chg, bool &bad)
{
    constexpr int U = 2;
    const int tid = threadIdx.x, W = blockDim.x, n = v.ndiff;
    for (int base = tid; base < n; base += U * W) {
        int2 e[U];
        bool ok[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int t = base + u * W;
            ok[u] = t < n;
            e[u] = v.diff(ok[u] ? t : n - 1);
        }
        int lbx[U], ubx[U], lby[U], uby[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int x = e[u].x & 0xffff, y = (uint32_t)e[u].x >> 16;
            lbx[u] = lds_ld(&lb[x]); ubx[u] = lds_ld(&ub[x]);
            lby[u] = lds_ld(&lb[y]); uby[u] = lds_ld(&ub[y]);
        }
        bool pu[U], pl[U], any = false;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int c = e[u].y;
            pu[u] = ok[u] && c + uby[u] < ubx[u];
            pl[u] = ok[u] && lbx[u] - c > lby[u];
            any |= pu[u] | pl[u];
        }
        if (any) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int x = e[u].x & 0xffff, y = (uint32_t)e[u].x >> 16, c = e[u].y;
                const int nu = c + uby[u], nl = lbx[u] - c;
                if (pu[u]) { join_ub(&ub[x], nu); chg = true; bad |= nu < lbx[u]; }
                if (pl[u]) { join_lb(&lb[y], nl); chg = true; bad |= nl > uby[u]; }
            }
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
template <bool DL>
__device__ __forceinline__ void sweep_reif(const View<DL> &v, int32_t *lb, int32_t *ub,
                                           bool &chg, bool &bad)
{
    constexpr int U = 4;
    constexpr int BIG = 0x3fffffff;
    const int tid = threadIdx.x, W = blockDim.x, n = v.nreif;
    for (int base = tid; base < n; base += U * W) {
        int2 e[U];
        bool ok[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int t = base + u * W;
            ok[u] = t < n;
            e[u] = v.reif(ok[u] ? t : n - 1);
        }
        int lbi[U], ubi[U], lbj[U], ubj[U], lbb[U], ubb[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int b = e[u].x & 0xffff, i = (uint32_t)e[u].x >> 16, j = e[u].y & 0xffff;
            lbi[u] = lds_ld(&lb[i]); ubi[u] = lds_ld(&ub[i]);
            lbj[u] = lds_ld(&lb[j]); ubj[u] = lds_ld(&ub[j]);
            lbb[u] = lds_ld(&lb[b]); ubb[u] = lds_ld(&ub[b]);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int d = e[u].y >> 16;
            const bool E1 = ubi[u] <= lbj[u];            // entailed(si <= sj)
            const bool E2 = ubj[u] <= lbi[u] + d - 1;    // entailed(sj < si + d)
            const bool on = lbb[u] >= 1, off = ubb[u] <= 0;
            const bool t_b1 = !on && E1 && E2;           // psi entailed: b >= 1
            const bool t_b0 = !off && (lbi[u] > ubj[u] || lbj[u] >= ubi[u] + d);  // not psi: b <= 0
            const bool o1 = off && E1, o2 = off && E2;
            const int nui = min(on ? ubj[u] : BIG, o1 ? ubj[u] - d : BIG);
            const int nlj = max(on ? lbi[u] : -BIG, o1 ? lbi[u] + d : -BIG);
            const int nuj = min(on ? ubi[u] + d - 1 : BIG, o2 ? ubi[u] - 1 : BIG);
            const int nli = max(on ? lbj[u] - d + 1 : -BIG, o2 ? lbj[u] + 1 : -BIG);
            const bool p_ui = nui < ubi[u], p_lj = nlj > lbj[u];
            const bool p_uj = nuj < ubj[u], p_li = nli > lbi[u];
            if (!ok[u] || !(t_b1 | t_b0 | p_ui | p_lj | p_uj | p_li))
                continue;
            const int b = e[u].x & 0xffff, i = (uint32_t)e[u].x >> 16, j = e[u].y & 0xffff;
            chg = true;
            if (t_b1) { join_lb(&lb[b], 1); bad |= ubb[u] < 1; }
            if (t_b0) { join_ub(&ub[b], 0); bad |= lbb[u] > 0; }
            if (p_ui) { join_ub(&ub[i], nui); bad |= nui < lbi[u]; }
            if (p_lj) { join_lb(&lb[j], nlj); bad |= nlj > ubj[u]; }
            if (p_uj) { join_ub(&ub[j], nuj); bad |= nuj < lbj[u]; }
            if (p_li) { join_lb(&lb[i], nli); bad |= nli > ubi[u]; }
        }
    }
}

// One term's tell of  a x <= rr  (rr = rhs - (S - m_t)) given the bounds the
// lane read for x: is it tighter, and the new bound.  Division only for
// |a| > 1 (floor toward -inf for a > 0, ceil toward +inf for a < 0).
__device__ __forceinline__ bool term_tight(int a, int lbx, int ubx, int rhs, int S)
{
    return a > 0 ? rhs - (S - a * lbx) < a * ubx : rhs - (S - a * ubx) < a * lbx;
}

__device__ __forceinline__ void term_tell(int32_t *lb, int32_t *ub, int x, int a, int lbx, int ubx,
                                          int rhs, int S, bool &chg, bool &bad)
{
    if (a > 0) {
        const int rr = rhs - (S - a * lbx);                 // a x <= rr
        const int nb = a == 1 ? rr : floor_div_pos(rr, a);
        join_ub(&ub[x], nb); chg = true; bad |= nb < lbx;
    } else {
        const int rr = rhs - (S - a * ubx);                 // x >= ceil(rr / a)
        const int nb = a == -1 ? -rr : -floor_div_pos(rr, -a);
        join_lb(&lb[x], nb); chg = true; bad |= nb > ubx;
    }
}

// kind 3: sum_t a_t x_t <= rhs.  A group of G lanes takes a row; lane l of
// the group holds terms first + l + G*k.  S (the sum of every term's
// smallest value, §2's lsum generalised) is a DPP sum over the group; each
// term is then told a_t x_t <= rhs - (S - m_t).  Rows are taken RR at a
// time per group; when every row fits in one chunk of TK terms per lane the
// tells use the bounds already in registers.
template <bool DL>
__device__ __forceinline__ void sweep_rows(const View<DL> &v, int32_t *lb, int32_t *ub,
                                           bool &chg, bool &bad)
{
    constexpr int RR = 4, TK = 2;
    const int tid = threadIdx.x, W = blockDim.x, n = v.nrows;
    if (n == 0) return;
    const int G = v.row_group, gl = tid & (G - 1), gid = tid / G, NG = W / G;
    const int KC = v.row_chunks;            // chunks of G terms in the longest row
    for (int rbase = gid; rbase < n; rbase += RR * NG) {
        int4 rd[RR];
        bool rok[RR];
#pragma unroll
        for (int q = 0; q < RR; ++q) {
            const int r = rbase + q * NG;
            rok[q] = r < n;
            rd[q] = v.rows(rok[q] ? r : n - 1);
        }
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
            int tl[RR][TK], tu[RR][TK];
#pragma unroll
            for (int q = 0; q < RR; ++q)
#pragma unroll
                for (int k = 0; k < TK; ++k) {
                    const int x = tv[q][k] & 0xffff;
                    tl[q][k] = lds_ld(&lb[x]);
                    tu[q][k] = lds_ld(&ub[x]);
                }
            int S[RR];
#pragma unroll
            for (int q = 0; q < RR; ++q) {
                int part = 0;
#pragma unroll
                for (int k = 0; k < TK; ++k) {
                    const int a = (int32_t)tv[q][k] >> 16;
                    part += tok[q][k] ? (a > 0 ? a * tl[q][k] : a * tu[q][k]) : 0;
                }
                S[q] = group_sum(part, G);
            }
            bool tight[RR][TK], any = false;
#pragma unroll
            for (int q = 0; q < RR; ++q)
#pragma unroll
                for (int k = 0; k < TK; ++k) {
                    tight[q][k] = tok[q][k] && term_tight((int32_t)tv[q][k] >> 16, tl[q][k],
                                                          tu[q][k], rd[q].z, S[q]);
                    any |= tight[q][k];
                }
            if (any) {
#pragma unroll
                for (int q = 0; q < RR; ++q)
#pragma unroll
                    for (int k = 0; k < TK; ++k)
                        if (tight[q][k])
                            term_tell(lb, ub, tv[q][k] & 0xffff, (int32_t)tv[q][k] >> 16,
                                      tl[q][k], tu[q][k], rd[q].z, S[q], chg, bad);
            }
        } else {
            // long rows: sum chunk by chunk, then tell chunk by chunk
            int S[RR];
#pragma unroll
            for (int q = 0; q < RR; ++q) S[q] = 0;
            for (int k = 0; k < KC; ++k) {
                const int o = gl + k * G;
#pragma unroll
                for (int q = 0; q < RR; ++q) {
                    if (rok[q] && o < rd[q].y) {
                        const uint32_t t = v.terms(rd[q].x + o);
                        const int x = t & 0xffff, a = (int32_t)t >> 16;
                        S[q] += a > 0 ? a * lds_ld(&lb[x]) : a * lds_ld(&ub[x]);
                    }
                }
            }
#pragma unroll
            for (int q = 0; q < RR; ++q) S[q] = group_sum(S[q], G);
            for (int k = 0; k < KC; ++k) {
                const int o = gl + k * G;
#pragma unroll
                for (int q = 0; q < RR; ++q) {
                    if (rok[q] && o < rd[q].y) {
                        const uint32_t t = v.terms(rd[q].x + o);
                        const int x = t & 0xffff, a = (int32_t)t >> 16;
                        // a bound re-read here can only have tightened since S
                        // was formed: the tell is then weaker, never unsound
                        const int lbx = lds_ld(&lb[x]), ubx = lds_ld(&ub[x]);
                        if (term_tight(a, lbx, ubx, rd[q].z, S[q]))
                            term_tell(lb, ub, x, a, lbx, ubx, rd[q].z, S[q], chg, bad);
                    }
                }
            }
        }
    }
}

// Fixed point of the LDS store (lb, ub) under every propagator of `v`.
// Returns 1 if the loop saw a failure, 0 at a fixed point (the post scan
// still has to look for an empty interval the loop did not see).
// Precondition: a barrier separates this call from any earlier read of the
// control words C_FLAG*, C_POSTFAIL, C_KEY.
template <bool DL>
__device__ int propagate_wg(const View<DL> &v, int32_t *lb, int32_t *ub, int32_t *ctl,
                            uint32_t &nsweeps)
{
    const int tid = threadIdx.x, lane = tid & 63;
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
        sweep_diff(v, lb, ub, chg, bad);
        sweep_reif(v, lb, ub, chg, bad);
        sweep_rows(v, lb, ub, chg, bad);
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

// ------------------------------------------------------ learned branching
// Features of decision variable q in the store (lb, ub) (x = dec[q], initial
// interval [lo, hi], H = max(1, hi - lo)):
//   f0 = (lb(x) - lo)/H, f1 = (ub(x) - lo)/H, f2 = (ub(x) - lb(x))/H,
//   f3 = degree share, f4 = min(1, min over rows x - y <= c of
//   (c + ub(y) - lb(x))/H), f5 = static load + (#reified items with si = x
//   and lb(b) >= 1) / N.
template <bool DL>
__device__ __forceinline__ void candidate_features(const View<DL> &v, int q, const int32_t *lb,
                                                   const int32_t *ub, float f[kNumFeat])
{
    const int x = v.dec(q);
    const float *st = v.fstat + 8 * (size_t)q;
    const int lo = __float_as_int(gread_f(st + 0));
    const float invH = gread_f(st + 1), degn = gread_f(st + 2), sl = gread_f(st + 3);
    const float invN = gread_f(st + 4);
    const int lbx = lds_ld(&lb[x]), ubx = lds_ld(&ub[x]);
    f[0] = (float)(lbx - lo) * invH;
    f[1] = (float)(ubx - lo) * invH;
    f[2] = (float)(ubx - lbx) * invH;
    f[3] = degn;
    float slack = 1.0f;
    const int r1 = gread(v.fr_ptr + q + 1);
    for (int k = gread(v.fr_ptr + q); k < r1; ++k) {
        const int2 e = gread(v.fr + k);
        slack = fminf(slack, (float)(e.y + lds_ld(&ub[e.x]) - lbx) * invH);
    }
    f[4] = slack;
    int cnt = 0;
    const int b1 = gread(v.fb_ptr + q + 1);
    for (int k = gread(v.fb_ptr + q); k < b1; ++k)
        cnt += lds_ld(&lb[gread(v.fb + k)]) >= 1;
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
// The store arrays are 16-byte aligned and padded to a multiple of 4
// variables; the pad holds lb = 0, ub = 0.
// With branching 2 (learned), `fsc` is an LDS scratch of 8 floats per
// decision variable and `ml` the lane's slice of the network.
template <bool DL>
__device__ void post_scan(const View<DL> &v, const int32_t *lb, const int32_t *ub, int32_t *ctl,
                          int branching, bool branch, float *fsc = nullptr,
                          const uint16_t *mlp = nullptr)
{
    const int tid = threadIdx.x, W = blockDim.x, lane = tid & 63;
    bool bad = false;
    const int nq = (v.nvars + 3) >> 2;
    const int4 *lb4 = reinterpret_cast<const int4 *>(lb);
    const int4 *ub4 = reinterpret_cast<const int4 *>(ub);
    for (int q = tid; q < nq; q += W) {
        const int4 l = lb4[q], u = ub4[q];
        bad |= (l.x > u.x) | (l.y > u.y) | (l.z > u.z) | (l.w > u.w);
    }
    unsigned long long key = ~0ull;
    if (branch && branching == 2) {
        // features of every unfixed candidate into LDS ...
        for (int q = tid; q < v.ndec; q += W) {
            const int x = v.dec(q);
            const bool open = lds_ld(&ub[x]) > lds_ld(&lb[x]);
            fsc[8 * q + 6] = open ? 1.f : 0.f;
            if (open) {
                float f[kNumFeat];
                candidate_features(v, q, lb, ub, f);
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

// ------------------------------------------------------ store copies
// The store of an instance with V variables occupies Vp = round_up(V, 4)
// entries of each array; entries V..Vp-1 hold (0, 0) so that quad-wise
// scans never see an empty interval there.

// lb/ub <- initial box (global, V entries), padding zeroed
__device__ __forceinline__ void load_box(int32_t *lb, int32_t *ub, const int32_t *lb0,
                                         const int32_t *ub0, int nvars)
{
    const int tid = threadIdx.x, W = blockDim.x, Vp = (nvars + 3) & ~3;
    for (int x = tid; x < Vp; x += W) {
        lb[x] = x < nvars ? gread(lb0 + x) : 0;
        ub[x] = x < nvars ? gread(ub0 + x) : 0;
    }
}

// copy Vp entries (16-byte aligned, quad-wise) from (slb, sub) to (dlb, dub);
// SG/DG: source/destination in global memory (else LDS)
template <bool SG, bool DG>
__device__ __forceinline__ void copy_store(int32_t *dlb, int32_t *dub, const int32_t *slb,
                                           const int32_t *sub, int nvars)
{
    const int tid = threadIdx.x, W = blockDim.x, nq = (nvars + 3) >> 2;
    for (int q = tid; q < nq; q += W) {
        const int4 l = SG ? gread(reinterpret_cast<const int4 *>(slb) + q)
                          : reinterpret_cast<const int4 *>(slb)[q];
        const int4 u = SG ? gread(reinterpret_cast<const int4 *>(sub) + q)
                          : reinterpret_cast<const int4 *>(sub)[q];
        if (DG) {
            gwrite4(reinterpret_cast<int4 *>(dlb) + q, l);
            gwrite4(reinterpret_cast<int4 *>(dub) + q, u);
        } else {
            reinterpret_cast<int4 *>(dlb)[q] = l;
            reinterpret_cast<int4 *>(dub)[q] = u;
        }
    }
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
    int32_t *lb = reinterpret_cast<int32_t *>(smem);
    int32_t *ub = lb + ((m.nvars + 3) & ~3);
    const View<false> v = view_global(m);
    for (int box = blockIdx.x; box < nbox; box += gridDim.x) {
        const size_t off = (size_t)box * m.nvars;
        load_box(lb, ub, lb_in + off, ub_in + off, m.nvars);
        lds_barrier();
        for (int q = tid; q < m.ndec; q += W) {
            float f[kNumFeat];
            candidate_features(v, q, lb, ub, f);
            for (int k = 0; k < kNumFeat; ++k)
                out[((size_t)box * m.ndec + q) * kNumFeat + k] = f[k];
        }
        lds_barrier();
    }
}

hipError_t launch_features(const DevModel *m_dev, int nvars, int nbox, const int32_t *lb_in,
                           const int32_t *ub_in, float *out, hipStream_t stream)
{
    const size_t lds = 2 * sizeof(int32_t) * (size_t)((nvars + 3) & ~3);
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
    const int tid = threadIdx.x, W = blockDim.x;
    int32_t *ctl = reinterpret_cast<int32_t *>(smem);
    int32_t *lb = ctl + kCtlWords;
    int32_t *ub = lb + ((m.nvars + 3) & ~3);
    char *dsc = reinterpret_cast<char *>(ub + ((m.nvars + 3) & ~3));
    View<DL> v;
    if constexpr (DL) v = stage_descriptors(m, dsc); else v = view_global(m);
    for (int box = blockIdx.x; box < nbox; box += gridDim.x) {
        const size_t off = (size_t)box * m.nvars;
        load_box(lb, ub, lb_in + off, ub_in + off, m.nvars);
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
// State only lane 0 uses lives in LDS (not in every lane's registers).
struct Lane0 {
    unsigned long long nodes, fails, sols, sweeps, don, maxd;
    unsigned long long since_flush, known_total, pf_qt, pf_qh;
    long long t_start;
    int32_t local_best, pf_best, pf_abort, pf_idle, idle_reg, pad;
};
static_assert(sizeof(Lane0) <= 4 * (kCtlWords - 32), "Lane0 must fit in the control block");

__device__ __forceinline__ int uni(int x) { return __builtin_amdgcn_readfirstlane(x); }

// lane 0: publish this workgroup's counters for instance `is`
__device__ void flush_counters(Lane0 &z, InstState *is, int mode)
{
    g_add(&is->nodes, z.nodes);
    g_add(&is->fails, z.fails);
    g_add(&is->sweeps, z.sweeps);
    g_add(&is->donations, z.don);
    g_add(&is->pops, 1ull);
    if (mode == 1) g_add(&is->solutions, z.sols);
    __hip_atomic_fetch_max(&is->max_depth, z.maxd, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    z.nodes = z.fails = z.sweeps = z.don = z.sols = z.maxd = 0;
}

// Persistent kernel: every workgroup loops { take a subtree record; DFS it }
// until the queue is empty and no subtree is in progress, or a limit hits.
template <bool DL, bool RL, bool LEARN>
__global__ __launch_bounds__(1024) void search_kernel(SearchParams P)
{
    extern __shared__ __align__(16) char smem[];
    const int tid = threadIdx.x, W = blockDim.x;
    const int Vp = (P.max_vars + 3) & ~3;
    int32_t *ctl = reinterpret_cast<int32_t *>(smem);
    Lane0 &z = *reinterpret_cast<Lane0 *>(ctl + 32);
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
    const bool learned = LEARN;   // the host picks this variant only with weights
    float *fsc = reinterpret_cast<float *>(reinterpret_cast<char *>(after) +
                                           align16(sizeof(int2) * (size_t)P.max_depth));
    char *dsc = reinterpret_cast<char *>(fsc) + (learned ? align16(32 * (size_t)P.max_ndec) : 0);
    const int branching = learned ? 2 : (P.branching == 1 ? 1 : 0);

    if (tid == 0) {
        z.nodes = z.fails = z.sols = z.sweeps = z.don = z.maxd = 0;
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
        }
        full_barrier();
        const long long pos = (long long)(((unsigned long long)(uint32_t)uni(ctl[C_SLOT_HI]) << 32) |
                                          (uint32_t)uni(ctl[C_SLOT]));
        if (pos < 0)
            break;
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        const int inst = uni(ctl[C_INST]);
        const int len = uni(ctl[C_LEN]);
        const int2 *rec = reinterpret_cast<const int2 *>(q_slot(P, (unsigned long long)pos) + 1);
        for (int i = tid; i < len; i += W) {
            const int2 dcs = gread(rec + i);
            stack[i] = make_int2(dcs.x & (0xffff | (int)kSideBit), dcs.y);
        }
        const DevModel &m = P.models[inst];
        if (inst != cur_inst) {
            if (tid == 0) z.local_best = INT32_MAX;
            if constexpr (DL) v = stage_descriptors(m, dsc); else v = view_global(m);
            cur_inst = inst;
        }
        const int nvars = m.nvars, ndec = m.ndec, objective = m.objective;
        load_box(lb, ub, m.lb0, m.ub0, nvars);
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
            z.pf_best = g_load(&is->best);
            z.pf_abort = 0;
        }
        // ---- depth-first search of this subtree
        for (;;) {
            if (tid == 0) {
                int stop = z.pf_abort != 0;
                if (P.node_limit > 0 && z.known_total + z.since_flush >= (unsigned long long)P.node_limit) {
                    g_store_rel(&P.g->abort, 1);
                    stop = 1;
                }
                if (P.t_limit_ticks > 0 && (long long)wall_clock64() - z.t_start > P.t_limit_ticks) {
                    g_store_rel(&P.g->abort, 2);
                    stop = 1;
                }
                if (P.cancel && (z.nodes & 255) == 0 && *P.cancel != 0) {
                    g_store_rel(&P.g->abort, 3);
                    stop = 1;
                }
                ctl[C_STOP] = stop;
                if (!stop && P.mode == 1) {
                    if (z.pf_best < z.local_best) z.local_best = z.pf_best;
                    if (z.local_best != INT32_MAX)
                        join_ub(&ub[objective], z.local_best - 1);
                }
                // loads consumed at the next node, so their latency overlaps
                // this node's propagation
                z.pf_best = g_load(&is->best);
                z.pf_abort = g_load(&P.g->abort);
                if (P.donate) {
                    z.pf_idle = g_load(&P.g->idle);
                    z.pf_qt = g_load(&P.g->q_tail);
                    z.pf_qh = g_load(&P.g->q_head);
                }
            }
            lds_barrier();
            if (uni(lds_ld(&ctl[C_STOP])))
                break;
            uint32_t nsw = 0;
            const int st = propagate_wg(v, lb, ub, ctl, nsw);
            post_scan(v, lb, ub, ctl, branching, st == 0, fsc, P.mlp);
            const int failed = uni(st | lds_ld(&ctl[C_POSTFAIL]));
            const unsigned long long key =
                *reinterpret_cast<volatile unsigned long long *>(ctl + C_KEY);
            if (tid == 0) {
                z.nodes += 1;
                z.since_flush += 1;
                z.sweeps += nsw;
                if ((unsigned long long)depth > z.maxd) z.maxd = depth;
                if (z.since_flush >= 256) {
                    z.known_total = g_add(&P.g->nodes_total, z.since_flush) + z.since_flush;
                    z.since_flush = 0;
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
                                P.sol_buf[(size_t)idx * ndec + q] = lb[v.dec(q)];
                        g_add(&is->sol_hash, solution_hash(lb, v, ndec));
                    } else {
                        const int32_t obj = lb[objective];
                        if (obj < z.local_best) z.local_best = obj;
                        const int32_t old = __hip_atomic_fetch_min(
                            &is->best, obj, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
                        if (obj < old) {
                            int32_t zz = 0;
                            while (!g_cas(&is->best_lock, zz, 1)) { zz = 0; __builtin_amdgcn_s_sleep(1); }
                            if (obj < is->pad[0]) {
                                for (int q = 0; q < ndec; ++q)
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
                    copy_store<false, !RL>(rlb, rub, lb, ub, nvars);
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
                    if (P.donate && z.pf_idle > 0 && z.pf_qt - z.pf_qh < (unsigned long long)z.pf_idle) {
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
                                z.don += 1;
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
            const int nd = uni(lds_ld(&ctl[C_DEPTH]));
            if (nd < 0) {
                finished = true;
                break;
            }
            depth = nd;
            // recompute: subtree root fixed point + decisions below it
            copy_store<!RL, false>(lb, ub, rlb, rub, nvars);
            lds_barrier();
            for (int i = depth0 + tid; i < depth; i += W)
                apply_decision(lb, ub, stack[i]);
            lds_barrier();
        }
        // ---- subtree done (or abandoned): publish counters
        if (tid == 0) {
            flush_counters(z, is, P.mode);
            if (finished) {
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

// ------------------------------------------------------------ MLP training
// Parameters (513 floats): W1[k][f] at k*6+f, b1 at 384+k, w2 at 448+k, b2
// at 512.  Score of a candidate: s = w2 . max(0, W1 x + b1) + b2, computed
// with one lane per hidden unit exactly as in the search (fmaf chain over
// the features, fixed-order wave sum).  Loss: mean over nodes of the
// cross-entropy between the target distribution over the node's candidates
// and the softmax of their scores.  Gradients are summed
// per wave into a partial row, then reduced in wave order (deterministic),
// fused with the Adam update and the bf16 copy the search reads.
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

// thread p: gradient p summed over the waves in order, then Adam
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

int mlp_partial_rows() { return 256 * 4; }   // waves of the training launches (256 x 256 threads)

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
    hipLaunchKernelGGL(mlp_reduce_adam_kernel, dim3((kNumParams + 1 + 255) / 256), dim3(256), 0,
                       stream, partial, blocks * 4, grad, params, m1, v1, wbf, lr, step, loss_dev);
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
size_t search_lds_bytes(int max_vars, int max_depth, size_t max_desc, bool desc_lds, bool root_lds,
                        int feat_ndec)
{
    const size_t Vp = (size_t)((max_vars + 3) & ~3);
    size_t b = sizeof(int32_t) * kCtlWords + 2 * Vp * sizeof(int32_t);
    if (root_lds) b += 2 * Vp * sizeof(int32_t);
    b += align16(sizeof(int2) * (size_t)max_depth);
    if (feat_ndec > 0) b += align16(32 * (size_t)feat_ndec);
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

// the search kernel variant for a layout and branching rule
static const void *search_fn(bool desc_lds, bool root_lds, bool learned)
{
#define PCCP_FN(a, b, c) reinterpret_cast<const void *>(search_kernel<a, b, c>)
    if (learned) {
        if (desc_lds && root_lds) return PCCP_FN(true, true, true);
        if (desc_lds) return PCCP_FN(true, false, true);
        if (root_lds) return PCCP_FN(false, true, true);
        return PCCP_FN(false, false, true);
    }
    if (desc_lds && root_lds) return PCCP_FN(true, true, false);
    if (desc_lds) return PCCP_FN(true, false, false);
    if (root_lds) return PCCP_FN(false, true, false);
    return PCCP_FN(false, false, false);
#undef PCCP_FN
}

hipError_t launch_search(const SearchParams &P, int grid, int block, size_t lds, bool desc_lds,
                         bool root_lds, hipStream_t stream)
{
    const int n = P.qcap > P.ninst ? P.qcap : P.ninst;
    hipLaunchKernelGGL(init_search_kernel, dim3((n + 255) / 256), dim3(256), 0, stream, P);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const void *fn = search_fn(desc_lds, root_lds, P.branching == 2 && P.mlp != nullptr);
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
                              bool desc_lds, bool root_lds, hipGraphExec_t *exec)
{
    const void *fn = search_fn(desc_lds, root_lds, P.branching == 2 && P.mlp != nullptr);
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

hipError_t search_occupancy(int block, size_t lds, bool desc_lds, bool root_lds, bool learned,
                            int *wgs_per_cu)
{
    const void *fn = search_fn(desc_lds, root_lds, learned);
    hipError_t e = set_lds_limit(fn, lds);
    if (e != hipSuccess) return e;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(wgs_per_cu, fn, block, lds);
}

}  // namespace pccp
