// Floating-point interval stores on gfx950: the lattices FInc and FDec of
// §2 (increasing / decreasing floats, ordered by the IEEE 754 total order of
// its footnote) and linear rows over the reals propagated with outward
// rounding (§6: intervals of reals approximated by intervals of floats).
//
// Store layout.  A bound is kept in LDS as its total-order key: the int32
// whose signed order is the IEEE total order of the float (the float's bits
// with the 31 magnitude bits flipped when the sign bit is set).  The join of
// FInc is then the LDS atomic max of the keys and the meet of FDec the
// atomic min, the same ds_max_i32 / ds_min_i32 as the integer store.  Zero
// bounds are canonical (-0 for a lower bound, +0 for an upper bound, the
// weaker zero of each lattice), so the total order of the keys agrees with
// the numeric order wherever the propagation compares bounds.
//
// Tells.  Term t of the row sum_u a_u x_u <= c gets
//   m_u  = a_u * (a_u > 0 ? lb : ub)(x_u)            rounded down
//   S_t  = sum of m_u over u != t, in term order from +0, each add rounded down
//   num  = c - S_t                                     rounded up
//   a_t > 0: ub(x_t) <- num / a_t rounded up;  a_t < 0: lb(x_t) <- num / a_t rounded down
// Each step is monotone in the store, so the tells are monotone and the
// least fixed point is reached by any fair schedule (§3 Theorem 2): the
// concurrent sweeps here give the same store, bit for bit, as a sequential
// loop.  One lane per row: the lane reads the bounds of the row's terms
// once, forms every m_u, and then runs the row's tells in term order,
// carrying the prefix m_0 + ... + m_{t-1} from one tell to the next, so
// S_t is that prefix followed by m_{t+1}, ..., m_{L-1}, the same additions
// in the same order as the definition.  Rows of up to kRowRegs terms keep
// their terms in registers, read from slot-major copies of the term tables
// (slot u of every row side by side, so a wavefront's reads of one slot are
// contiguous); longer rows read the row-major tables term by term.  The
// additions and products rounded down run on the hardware adder and
// multiplier with the MODE register's f32 rounding field switched for them
// (IEEE arithmetic, exact up to that one rounding); c - S_t rounded up is
// the negation of S_t - c rounded down; the quotients are rounded as
// quot_out below explains.
//
// Fixed point and failure (§5): per-wavefront ballots of the change and
// failure bits into three rotating LDS words, one barrier per sweep, and a
// scan of the store at the end.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/pccp.h"
#include "pccp_launch.h"

namespace pccp {
namespace {

// total-order key of a float and back (an involution on the bits)
__host__ __device__ inline int32_t fkey(float f)
{
    uint32_t b;
    memcpy(&b, &f, 4);
    b ^= (uint32_t)((int32_t)b >> 31) & 0x7fffffffu;
    return (int32_t)b;
}
__host__ __device__ inline float fval(int32_t k)
{
    uint32_t b = (uint32_t)k;
    b ^= (uint32_t)(k >> 31) & 0x7fffffffu;
    float f;
    memcpy(&f, &b, 4);
    return f;
}
__host__ __device__ inline float canon_lb(float v) { return v == 0.0f ? -0.0f : v; }
__host__ __device__ inline float canon_ub(float v) { return v == 0.0f ? 0.0f : v; }

// The quotient x = num / a rounded up (a > 0) or down (a < 0), from
// inv = 1 / a rounded to nearest in double precision.
//  - q = num * inv (double) is within 2^-52 of x, relatively; a quotient of
//    two floats that is not itself a float lies at least 2^-48 of its size
//    from every float (num - g a is a nonzero multiple of the last place of
//    the 48-bit product g a), so f = q rounded to float is x's float
//    neighbour below or above (x itself when x is a float).
//  - r = num - f a is exact in one fma (f a has 48 bits and num lines up
//    with its top bits), and r = a (x - f): for a > 0, r > 0 says x > f and
//    the quotient rounded up is the float above f; for a < 0, r > 0 says
//    x < f and the quotient rounded down is the float below f.
// Infinite num (an infinite sum of the other terms) gives an infinite f
// and r NaN, left as is; zero num gives a zero f of the quotient's sign.
// The step to the neighbour works on the bits: away from zero adds one,
// toward zero takes one off (from an infinity this gives the largest finite
// float, the only step that can arise there), and from a zero it gives the
// smallest subnormal of the direction's sign.
__device__ __forceinline__ float quot_out(float num, float a, double inv)
{
    const float f = (float)((double)num * inv);
    const bool step = fma(-(double)f, (double)a, (double)num) > 0.0;
    const bool up = a > 0.0f;
    const uint32_t b = __float_as_uint(f);
    uint32_t nb = (f > 0.0f) == up ? b + 1u : b - 1u;
    nb = f == 0.0f ? (up ? 1u : 0x80000001u) : nb;
    return step ? __uint_as_float(nb) : f;
}

// Rows of at most this many terms keep their terms in registers.
constexpr int kRowRegs = 8;   // frow's dispatch covers lengths 1..8

struct FDev {
    int32_t nvars, nrows, nterms, pad;
    const int2 *rowd;       // {first term, number of terms}
    const float *rhs;
    const int32_t *tvar;    // variable of each term, row-major
    const float *tcoef;     // coefficient of each term, row-major
    const int32_t *svar;    // slot-major: svar[u * nrows + r] = variable of term u of row r
    const float *scoef;     // slot-major coefficients (rows of up to kRowRegs terms)
    const double *sinv;     // slot-major 1 / coefficient, rounded to nearest in double
};

// Directed rounding.  The f32 rounding field of the MODE register (bits 1:0;
// 0 to nearest, the kernel's default, 2 toward -inf) is switched to toward
// -inf around a short run of additions, subtractions or products and put
// back after it, all inside one asm statement, so the compiler can move no
// other float instruction into the run.  Two wait states separate a write of
// MODE from the next one (the s_nop after the restoring write, and the
// VALU instruction plus s_nop 0 before it).
#define PCCP_RD_ON "s_setreg_imm32_b32 hwreg(HW_REG_MODE, 0, 2), 2\n\t"
#define PCCP_RD_OFF "s_nop 0\n\ts_setreg_imm32_b32 hwreg(HW_REG_MODE, 0, 2), 0\n\ts_nop 1"

__device__ __forceinline__ float add_rd(float a, float b)
{
    float r;
    asm volatile(PCCP_RD_ON "v_add_f32 %0, %1, %2\n\t" PCCP_RD_OFF : "=&v"(r) : "v"(a), "v"(b));
    return r;
}
__device__ __forceinline__ float mul_rd(float a, float b)
{
    float r;
    asm volatile(PCCP_RD_ON "v_mul_f32 %0, %1, %2\n\t" PCCP_RD_OFF : "=&v"(r) : "v"(a), "v"(b));
    return r;
}
// two products rounded down under one switch of the rounding mode
__device__ __forceinline__ void mul2_rd(float a0, float b0, float a1, float b1, float &r0, float &r1)
{
    asm volatile(PCCP_RD_ON "v_mul_f32 %0, %2, %3\n\t"
                 "v_mul_f32 %1, %4, %5\n\t" PCCP_RD_OFF
                 : "=&v"(r0), "=&v"(r1) : "v"(a0), "v"(b0), "v"(a1), "v"(b1));
}
// c - s rounded up, as the negation of s - c rounded down
__device__ __forceinline__ float sub_ru(float c, float s)
{
    float r;
    asm volatile(PCCP_RD_ON "v_sub_f32 %0, %1, %2\n\t" PCCP_RD_OFF : "=&v"(r) : "v"(s), "v"(c));
    return -r;
}

// The rounded-down part of term t's tell with K = L - 1 - t terms after it,
// under one switch of the rounding mode:
//   S     = pre + ms[0] + ... + ms[K-1]     (pre = m_0 + ... + m_{t-1}; ms[k] = m_{t+1+k})
//   nneg  = S - c                           (so c - S rounded up is -nneg)
//   pre'  = pre + m_t                       (K > 0 only: the next term's prefix)
// each operation rounded toward -inf, in this order.
#define PCCP_CH(n) "v_add_f32 %2, %2, %" #n "\n\t"
#define PCCP_TAIL "v_sub_f32 %0, %2, %4\n\t" "v_add_f32 %1, %3, %5\n\t" PCCP_RD_OFF
#define PCCP_MS(k) , "v"(ms[k])
template <int K>
__device__ __forceinline__ void rd_tell(float pre, float c, float mt, const float *ms, float &nneg,
                                        float &pre_next)
{
    float S;
    if constexpr (K == 0) {
        asm volatile(PCCP_RD_ON "v_sub_f32 %0, %1, %2\n\t" PCCP_RD_OFF : "=&v"(nneg) : "v"(pre), "v"(c));
        pre_next = pre;
    } else if constexpr (K == 1) {
        asm volatile(PCCP_RD_ON "v_add_f32 %2, %3, %6\n\t" PCCP_TAIL
                     : "=&v"(nneg), "=&v"(pre_next), "=&v"(S) : "v"(pre), "v"(c), "v"(mt) PCCP_MS(0));
    } else if constexpr (K == 2) {
        asm volatile(PCCP_RD_ON "v_add_f32 %2, %3, %6\n\t" PCCP_CH(7) PCCP_TAIL
                     : "=&v"(nneg), "=&v"(pre_next), "=&v"(S)
                     : "v"(pre), "v"(c), "v"(mt) PCCP_MS(0) PCCP_MS(1));
    } else if constexpr (K == 3) {
        asm volatile(PCCP_RD_ON "v_add_f32 %2, %3, %6\n\t" PCCP_CH(7) PCCP_CH(8) PCCP_TAIL
                     : "=&v"(nneg), "=&v"(pre_next), "=&v"(S)
                     : "v"(pre), "v"(c), "v"(mt) PCCP_MS(0) PCCP_MS(1) PCCP_MS(2));
    } else if constexpr (K == 4) {
        asm volatile(PCCP_RD_ON "v_add_f32 %2, %3, %6\n\t" PCCP_CH(7) PCCP_CH(8) PCCP_CH(9) PCCP_TAIL
                     : "=&v"(nneg), "=&v"(pre_next), "=&v"(S)
                     : "v"(pre), "v"(c), "v"(mt) PCCP_MS(0) PCCP_MS(1) PCCP_MS(2) PCCP_MS(3));
    } else if constexpr (K == 5) {
        asm volatile(PCCP_RD_ON "v_add_f32 %2, %3, %6\n\t" PCCP_CH(7) PCCP_CH(8) PCCP_CH(9) PCCP_CH(10)
                     PCCP_TAIL
                     : "=&v"(nneg), "=&v"(pre_next), "=&v"(S)
                     : "v"(pre), "v"(c), "v"(mt) PCCP_MS(0) PCCP_MS(1) PCCP_MS(2) PCCP_MS(3) PCCP_MS(4));
    } else if constexpr (K == 6) {
        asm volatile(PCCP_RD_ON "v_add_f32 %2, %3, %6\n\t" PCCP_CH(7) PCCP_CH(8) PCCP_CH(9) PCCP_CH(10)
                     PCCP_CH(11) PCCP_TAIL
                     : "=&v"(nneg), "=&v"(pre_next), "=&v"(S)
                     : "v"(pre), "v"(c), "v"(mt) PCCP_MS(0) PCCP_MS(1) PCCP_MS(2) PCCP_MS(3) PCCP_MS(4)
                       PCCP_MS(5));
    } else {
        static_assert(K == 7, "rows of at most 8 terms");
        asm volatile(PCCP_RD_ON "v_add_f32 %2, %3, %6\n\t" PCCP_CH(7) PCCP_CH(8) PCCP_CH(9) PCCP_CH(10)
                     PCCP_CH(11) PCCP_CH(12) PCCP_TAIL
                     : "=&v"(nneg), "=&v"(pre_next), "=&v"(S)
                     : "v"(pre), "v"(c), "v"(mt) PCCP_MS(0) PCCP_MS(1) PCCP_MS(2) PCCP_MS(3) PCCP_MS(4)
                       PCCP_MS(5) PCCP_MS(6));
    }
}

__device__ __forceinline__ void fbarrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

__device__ __forceinline__ int2 fdom(const int2 *st, int x)
{
    const unsigned long long u =
        __hip_atomic_load(reinterpret_cast<unsigned long long *>(const_cast<int2 *>(st + x)),
                          __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    return make_int2((int32_t)(uint32_t)u, (int32_t)(uint32_t)(u >> 32));
}

// the bound that term a x contributes at its least: a lb(x) for a > 0, a ub(x) otherwise
__device__ __forceinline__ float fside(float a, int2 d) { return fval(a > 0.0f ? d.x : d.y); }
__device__ __forceinline__ float fterm(float a, int2 d) { return mul_rd(a, fside(a, d)); }

// The tell of one term: num = c - S_t rounded up, dx the bounds of x read
// before the row's tells (bounds only tighten, so a stale dx can only report
// a change that another lane made first, never miss one; a failure it
// misses is found by the scan at the end).
__device__ __forceinline__ void ftell(int2 *st, float num, float a, double inv, int x, int2 dx,
                                      bool &chg, bool &bad)
{
    const float b = quot_out(num, a, inv);
    if (a > 0.0f) {
        const int32_t k = fkey(canon_ub(b));
        if (k < dx.y) {
            __hip_atomic_fetch_min(&st[x].y, k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            chg = true;
            bad |= k < dx.x;
        }
    } else {
        const int32_t k = fkey(canon_lb(b));
        if (k > dx.x) {
            __hip_atomic_fetch_max(&st[x].x, k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            chg = true;
            bad |= k > dx.y;
        }
    }
}

// The tells of terms T.. of a row of N terms, pre = m_0 + ... + m_{T-1}
// rounded down (+0 for T = 0).
template <int N, int T>
__device__ __forceinline__ void frow_tells(int2 *st, float c, const float *av, const float *mv,
                                           const double *iv, const int *xv, const int2 *dv, float pre,
                                           bool &chg, bool &bad)
{
    if constexpr (T < N) {
        float nneg, pn;
        rd_tell<N - 1 - T>(pre, c, mv[T], mv + T + 1, nneg, pn);
        ftell(st, -nneg, av[T], iv[T], xv[T], dv[T], chg, bad);
        frow_tells<N, T + 1>(st, c, av, mv, iv, xv, dv, pn, chg, bad);
    }
}

// A row of exactly N terms held in registers (slot u of row r at u * nrows + r
// of the slot-major tables), every lane of the wavefront on a row of N terms.
template <int N>
__device__ __forceinline__ void frow_exact(const FDev &m, int2 *st, int r, float c, bool &chg, bool &bad)
{
    float av[N], mv[N], sv[N];
    double iv[N];
    int xv[N];
    int2 dv[N];
#pragma unroll
    for (int u = 0; u < N; ++u) {
        const int o = u * m.nrows + r;
        av[u] = m.scoef[o];
        iv[u] = m.sinv[o];
        xv[u] = m.svar[o];
        dv[u] = fdom(st, xv[u]);
        sv[u] = fside(av[u], dv[u]);
    }
#pragma unroll
    for (int u = 0; u + 1 < N; u += 2) mul2_rd(av[u], sv[u], av[u + 1], sv[u + 1], mv[u], mv[u + 1]);
    if constexpr (N % 2 == 1) mv[N - 1] = mul_rd(av[N - 1], sv[N - 1]);
    frow_tells<N, 0>(st, c, av, mv, iv, xv, dv, 0.0f, chg, bad);
}

// A row of L <= kRowRegs terms in a wavefront whose rows differ in length:
// the same operations, one switch of the rounding mode each.
__device__ __forceinline__ void frow_mixed(const FDev &m, int2 *st, int r, int L, float c, bool &chg,
                                           bool &bad)
{
    float av[kRowRegs], mv[kRowRegs];
    double iv[kRowRegs];
    int xv[kRowRegs];
    int2 dv[kRowRegs];
#pragma unroll
    for (int u = 0; u < kRowRegs; ++u) {
        av[u] = 1.0f;
        iv[u] = 1.0;
        mv[u] = 0.0f;
        xv[u] = 0;
        dv[u] = make_int2(0, 0);
        if (u < L) {
            const int o = u * m.nrows + r;
            av[u] = m.scoef[o];
            iv[u] = m.sinv[o];
            xv[u] = m.svar[o];
            dv[u] = fdom(st, xv[u]);
            mv[u] = fterm(av[u], dv[u]);
        }
    }
    float pre = 0.0f;
#pragma unroll
    for (int t = 0; t < kRowRegs; ++t) {
        if (t < L) {
            float s = pre;
#pragma unroll
            for (int u = t + 1; u < kRowRegs; ++u)
                if (u < L) s = add_rd(s, mv[u]);
            ftell(st, sub_ru(c, s), av[t], iv[t], xv[t], dv[t], chg, bad);
            pre = add_rd(pre, mv[t]);
        }
    }
}

// One sweep of the tells of row r.  The host orders the rows by their
// number of terms, so a wavefront's 64 consecutive rows nearly always share
// it and take the code compiled for that length.
__device__ __forceinline__ void frow(const FDev &m, int2 *st, int r, bool &chg, bool &bad)
{
    const int2 rd = m.rowd[r];
    const float c = m.rhs[r];
    const int lw = __builtin_amdgcn_readfirstlane(rd.y);
    if (lw <= kRowRegs && __all(rd.y == lw)) {
        switch (lw) {
        case 1: frow_exact<1>(m, st, r, c, chg, bad); break;
        case 2: frow_exact<2>(m, st, r, c, chg, bad); break;
        case 3: frow_exact<3>(m, st, r, c, chg, bad); break;
        case 4: frow_exact<4>(m, st, r, c, chg, bad); break;
        case 5: frow_exact<5>(m, st, r, c, chg, bad); break;
        case 6: frow_exact<6>(m, st, r, c, chg, bad); break;
        case 7: frow_exact<7>(m, st, r, c, chg, bad); break;
        default: frow_exact<8>(m, st, r, c, chg, bad); break;
        }
        return;
    }
    if (rd.y <= kRowRegs) {
        frow_mixed(m, st, r, rd.y, c, chg, bad);
        return;
    }
    // a long row, term by term from the row-major tables
    float pre = 0.0f;
    for (int t = rd.x; t < rd.x + rd.y; ++t) {
        const float a = m.tcoef[t];
        const int x = m.tvar[t];
        const int2 dx = fdom(st, x);
        float s = pre;
        for (int u = t + 1; u < rd.x + rd.y; ++u) s = add_rd(s, fterm(m.tcoef[u], fdom(st, m.tvar[u])));
        ftell(st, sub_ru(c, s), a, 1.0 / (double)a, x, dx, chg, bad);
        pre = add_rd(pre, fterm(a, dx));
    }
}

// One workgroup per box; status 0 fixed point, 1 failed.
__global__ __launch_bounds__(1024) void fpropagate_batch_kernel(FDev m, int nbox, const float *lb_in,
                                                                const float *ub_in, float *lb_out,
                                                                float *ub_out, int32_t *status,
                                                                int32_t *sweeps)
{
    extern __shared__ __align__(16) char smem[];
    int32_t *ctl = reinterpret_cast<int32_t *>(smem);
    int2 *st = reinterpret_cast<int2 *>(smem + 16);
    const int tid = threadIdx.x, lane = tid & 63, W = blockDim.x;
    for (int box = blockIdx.x; box < nbox; box += gridDim.x) {
        const size_t off = (size_t)box * m.nvars;
        for (int x = tid; x < m.nvars; x += W)
            st[x] = make_int2(fkey(canon_lb(lb_in[off + x])), fkey(canon_ub(ub_in[off + x])));
        if (tid == 0) {
            ctl[0] = 0;
            ctl[1] = 0;
            ctl[2] = 0;
            ctl[3] = 0;
        }
        fbarrier();
        int slot = 0, nsw = 0, failed = 0;
        for (;;) {
            bool chg = false, bad = false;
            for (int r = tid; r < m.nrows; r += W) frow(m, st, r, chg, bad);
            const int flags = (__any(chg) ? 1 : 0) | (__any(bad) ? 2 : 0);
            if (lane == 0 && flags)
                __hip_atomic_fetch_or(&ctl[slot], flags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            const int next = slot == 2 ? 0 : slot + 1;
            if (tid == 0) ctl[next] = 0;
            fbarrier();
            ++nsw;
            const int f = __hip_atomic_load(&ctl[slot], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            if (f & 2) { failed = 1; break; }
            if (!(f & 1)) break;
            slot = next;
        }
        // the failure scan: an empty interval the loop did not flag
        bool empty = false;
        for (int x = tid; x < m.nvars; x += W) {
            const int2 d = st[x];
            empty |= d.x > d.y;
        }
        if (__any(empty) && lane == 0)
            __hip_atomic_fetch_or(&ctl[3], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        fbarrier();
        failed |= __hip_atomic_load(&ctl[3], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        for (int x = tid; x < m.nvars; x += W) {
            const int2 d = st[x];
            lb_out[off + x] = fval(d.x);
            ub_out[off + x] = fval(d.y);
        }
        if (tid == 0) {
            status[box] = failed;
            if (sweeps) sweeps[box] = nsw;
        }
        fbarrier();
    }
}

}  // namespace
}  // namespace pccp

using namespace pccp;

// ------------------------------------------------------------------ host side
struct pccp_fmodel {
    std::vector<float> lb, ub;
    std::vector<int32_t> row_ptr{0}, var;
    std::vector<float> coef, rhs;
};

struct pccp_fsolver {
    int device = 0;
    hipStream_t stream = nullptr;
    int32_t wg_size = 256;
    int32_t nvars = 0, nrows = 0, nterms = 0;
    void *tables = nullptr;
    FDev dev{};
    size_t lds_max = 0;
    int num_cus = 0;
};

#define FHIPCHK(call)                                                                       \
    do {                                                                                    \
        hipError_t e_ = (call);                                                             \
        if (e_ != hipSuccess)                                                               \
            return internal_fail(PCCP_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

extern "C" int32_t pccp_fmodel_create(pccp_fmodel **out)
{
    if (!out) return internal_fail(PCCP_E_INVALID_ARG, "pccp_fmodel_create: out is NULL");
    *out = new (std::nothrow) pccp_fmodel();
    return *out ? PCCP_OK : internal_fail(PCCP_E_NOMEM, "pccp_fmodel_create: out of memory");
}

extern "C" int32_t pccp_fmodel_destroy(pccp_fmodel *m)
{
    delete m;
    return PCCP_OK;
}

extern "C" int32_t pccp_fmodel_add_vars(pccp_fmodel *m, int32_t n, const float *lb, const float *ub,
                                        int32_t *first_id)
{
    if (!m || n < 0 || (n > 0 && (!lb || !ub)))
        return internal_fail(PCCP_E_INVALID_ARG, "pccp_fmodel_add_vars: bad arguments");
    if ((int64_t)m->lb.size() + n > kMaxVars)
        return internal_fail(PCCP_E_UNSUPPORTED, "pccp_fmodel_add_vars: more than 65535 variables");
    if (first_id) *first_id = (int32_t)m->lb.size();
    m->lb.insert(m->lb.end(), lb, lb + n);
    m->ub.insert(m->ub.end(), ub, ub + n);
    return PCCP_OK;
}

extern "C" int32_t pccp_fmodel_add_linear_le(pccp_fmodel *m, int32_t nterms, const float *coef,
                                             const int32_t *var, float rhs)
{
    if (!m || nterms < 1 || !coef || !var)
        return internal_fail(PCCP_E_INVALID_ARG, "pccp_fmodel_add_linear_le: bad arguments");
    m->coef.insert(m->coef.end(), coef, coef + nterms);
    m->var.insert(m->var.end(), var, var + nterms);
    m->rhs.push_back(rhs);
    m->row_ptr.push_back((int32_t)m->coef.size());
    return PCCP_OK;
}

extern "C" int32_t pccp_fsolver_create(const pccp_fmodel *m, int32_t wg_size, void *stream,
                                       pccp_fsolver **out)
{
    if (!m || !out) return internal_fail(PCCP_E_INVALID_ARG, "pccp_fsolver_create: bad arguments");
    *out = nullptr;
    if (wg_size == 0) wg_size = 256;
    if (wg_size < 64 || wg_size > kMaxWg || wg_size % 64 != 0)
        return internal_fail(PCCP_E_INVALID_ARG, "pccp_fsolver_create: wg_size must be a multiple of 64 and <= 1024");
    const int32_t V = (int32_t)m->lb.size(), R = (int32_t)m->rhs.size();
    const int32_t T = (int32_t)m->coef.size();
    for (int32_t v = 0; v < V; ++v)
        if (!std::isfinite(m->lb[v]) || !std::isfinite(m->ub[v]))
            return internal_fail(PCCP_E_MODEL, "variable " + std::to_string(v) + ": bounds must be finite");
    std::vector<char> seen(V > 0 ? V : 1, 0);
    // rows in order of their number of terms (stable), so that a wavefront's
    // rows share one length; any order of the rows reaches the same fixed point
    std::vector<int32_t> order(R);
    for (int32_t r = 0; r < R; ++r) order[r] = r;
    std::stable_sort(order.begin(), order.end(), [&](int32_t p, int32_t q) {
        return m->row_ptr[p + 1] - m->row_ptr[p] < m->row_ptr[q + 1] - m->row_ptr[q];
    });
    std::vector<float> rhs(R);
    std::vector<int2> rowd(R);
    // slot-major copies for rows of up to kRowRegs terms (zero where a row is shorter)
    std::vector<int32_t> svar((size_t)kRowRegs * R, 0);
    std::vector<float> scoef((size_t)kRowRegs * R, 0.0f);
    std::vector<double> sinv((size_t)kRowRegs * R, 1.0);
    for (int32_t i = 0; i < R; ++i) {
        const int32_t r = order[i], a0 = m->row_ptr[r], a1 = m->row_ptr[r + 1];
        if (!std::isfinite(m->rhs[r]))
            return internal_fail(PCCP_E_MODEL, "row " + std::to_string(r) + ": right-hand side must be finite");
        for (int32_t t = a0; t < a1; ++t) {
            const int32_t x = m->var[t];
            if (x < 0 || x >= V) return internal_fail(PCCP_E_MODEL, "row " + std::to_string(r) + ": variable out of range");
            if (!std::isfinite(m->coef[t]) || m->coef[t] == 0.0f)
                return internal_fail(PCCP_E_MODEL, "row " + std::to_string(r) + ": coefficient zero or not finite");
            if (seen[x]) return internal_fail(PCCP_E_MODEL, "row " + std::to_string(r) + ": variable repeated");
            seen[x] = 1;
            if (a1 - a0 <= kRowRegs) {
                svar[(size_t)(t - a0) * R + i] = x;
                scoef[(size_t)(t - a0) * R + i] = m->coef[t];
                sinv[(size_t)(t - a0) * R + i] = 1.0 / (double)m->coef[t];
            }
        }
        for (int32_t t = a0; t < a1; ++t) seen[m->var[t]] = 0;
        rowd[i] = make_int2(a0, a1 - a0);
        rhs[i] = m->rhs[r];
    }
    pccp_fsolver *s = new (std::nothrow) pccp_fsolver();
    if (!s) return internal_fail(PCCP_E_NOMEM, "pccp_fsolver_create: out of memory");
    s->stream = reinterpret_cast<hipStream_t>(stream);
    s->wg_size = wg_size;
    s->nvars = V;
    s->nrows = R;
    s->nterms = T;
    hipDeviceProp_t prop;
    hipError_t e = hipGetDevice(&s->device);
    if (e == hipSuccess) e = hipGetDeviceProperties(&prop, s->device);
    if (e != hipSuccess) {
        delete s;
        return internal_fail(PCCP_E_DEVICE, std::string("device query: ") + hipGetErrorString(e));
    }
    s->lds_max = prop.sharedMemPerBlock;
    s->num_cus = prop.multiProcessorCount;
    if (16 + 8 * (size_t)V > s->lds_max) {
        delete s;
        return internal_fail(PCCP_E_LDS_CAPACITY, "the float store (8 bytes per variable) does not fit in LDS");
    }
    auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
    const size_t o_rowd = 0, o_rhs = o_rowd + al(8 * (size_t)R), o_tvar = o_rhs + al(4 * (size_t)R);
    const size_t o_tcoef = o_tvar + al(4 * (size_t)T), o_svar = o_tcoef + al(4 * (size_t)T);
    const size_t o_scoef = o_svar + al(4 * (size_t)kRowRegs * R);
    const size_t o_sinv = o_scoef + al(4 * (size_t)kRowRegs * R);
    const size_t total = o_sinv + al(8 * (size_t)kRowRegs * R) + 256;
    std::vector<char> host(total, 0);
    if (R) {
        memcpy(host.data() + o_rowd, rowd.data(), 8 * (size_t)R);
        memcpy(host.data() + o_rhs, rhs.data(), 4 * (size_t)R);
        memcpy(host.data() + o_svar, svar.data(), 4 * (size_t)kRowRegs * R);
        memcpy(host.data() + o_scoef, scoef.data(), 4 * (size_t)kRowRegs * R);
        memcpy(host.data() + o_sinv, sinv.data(), 8 * (size_t)kRowRegs * R);
    }
    if (T) {
        memcpy(host.data() + o_tvar, m->var.data(), 4 * (size_t)T);
        memcpy(host.data() + o_tcoef, m->coef.data(), 4 * (size_t)T);
    }
    e = hipMalloc(&s->tables, total);
    if (e == hipSuccess) e = hipMemcpyAsync(s->tables, host.data(), total, hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) {
        if (s->tables) (void)hipFree(s->tables);
        delete s;
        return internal_fail(PCCP_E_DEVICE, std::string("upload: ") + hipGetErrorString(e));
    }
    char *base = reinterpret_cast<char *>(s->tables);
    s->dev.nvars = V;
    s->dev.nrows = R;
    s->dev.nterms = T;
    s->dev.rowd = reinterpret_cast<const int2 *>(base + o_rowd);
    s->dev.rhs = reinterpret_cast<const float *>(base + o_rhs);
    s->dev.tvar = reinterpret_cast<const int32_t *>(base + o_tvar);
    s->dev.tcoef = reinterpret_cast<const float *>(base + o_tcoef);
    s->dev.svar = reinterpret_cast<const int32_t *>(base + o_svar);
    s->dev.scoef = reinterpret_cast<const float *>(base + o_scoef);
    s->dev.sinv = reinterpret_cast<const double *>(base + o_sinv);
    *out = s;
    return PCCP_OK;
}

extern "C" int32_t pccp_fsolver_destroy(pccp_fsolver *s)
{
    if (!s) return PCCP_OK;
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(s->device);
    (void)hipStreamSynchronize(s->stream);
    if (s->tables) (void)hipFree(s->tables);
    (void)hipSetDevice(prev);
    delete s;
    return PCCP_OK;
}

extern "C" int32_t pccp_fpropagate_batch(pccp_fsolver *s, int32_t nbox, const float *lb_in,
                                         const float *ub_in, float *lb_out, float *ub_out,
                                         int32_t *status, int32_t *sweeps)
{
    if (!s || nbox < 0 || (nbox > 0 && (!lb_in || !ub_in || !lb_out || !ub_out || !status)))
        return internal_fail(PCCP_E_INVALID_ARG, "pccp_fpropagate_batch: bad arguments");
    if (nbox == 0) return PCCP_OK;
    const size_t lds = 16 + 8 * (size_t)((s->nvars + 1) & ~1);
    const int grid = std::min(nbox, std::max(1, s->num_cus * 8));
    FHIPCHK(hipSetDevice(s->device));
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(fpropagate_batch_kernel),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    (void)hipGetLastError();
    hipLaunchKernelGGL(fpropagate_batch_kernel, dim3(grid), dim3(s->wg_size), lds, s->stream, s->dev,
                       nbox, lb_in, ub_in, lb_out, ub_out, status, sweeps);
    FHIPCHK(hipGetLastError());
    return PCCP_OK;
}
