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
// loop.  One lane per term; a row's terms are read in order by each of its
// lanes.  The directed roundings are the device library's correctly rounded
// additions and products in the rounding mode asked for; the quotients are
// rounded as div_rd / div_ru below explain.
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

extern "C" __device__ float __ocml_add_rtn_f32(float, float);
extern "C" __device__ float __ocml_sub_rtp_f32(float, float);
extern "C" __device__ float __ocml_mul_rtn_f32(float, float);

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

// The quotient of two floats rounded down / up.  The quotient is formed in
// double precision (round to nearest) and then rounded to float in the
// direction asked for: a quotient of two 24-bit significands that is not
// itself a float lies at least 2^-48 of its size away from every float,
// farther than the double's rounding error (2^-53), so the double falls on
// the same side of every float as the exact quotient and the directed
// conversion of the double is the directed rounding of the exact quotient.
__device__ __forceinline__ float next_down(float f)
{
    if (f != f || f == -INFINITY) return f;
    if (f == 0.0f) return -1.40129846e-45f;              // the largest negative float
    uint32_t b = __float_as_uint(f);
    b = f > 0.0f ? b - 1u : b + 1u;
    return __uint_as_float(b);
}
__device__ __forceinline__ float next_up(float f) { return -next_down(-f); }
__device__ __forceinline__ float div_rd(float a, float b)
{
    const double q = (double)a / (double)b;
    const float f = (float)q;
    return (double)f > q ? next_down(f) : f;
}
__device__ __forceinline__ float div_ru(float a, float b)
{
    const double q = (double)a / (double)b;
    const float f = (float)q;
    return (double)f < q ? next_up(f) : f;
}

struct FDev {
    int32_t nvars, nrows, nterms, pad;
    const int2 *rowd;       // {first term, number of terms}
    const float *rhs;
    const int32_t *tvar;    // variable of each term
    const float *tcoef;     // coefficient of each term
    const int32_t *trow;    // row of each term
};

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
            for (int t0 = __builtin_amdgcn_readfirstlane(tid - lane); t0 < m.nterms; t0 += W) {
                const int t = t0 + lane;
                if (t >= m.nterms) continue;
                const int r = m.trow[t];
                const int2 rd = m.rowd[r];
                float s = 0.0f;
                for (int u = rd.x; u < rd.x + rd.y; ++u) {
                    if (u == t) continue;
                    const float a = m.tcoef[u];
                    const int2 d = fdom(st, m.tvar[u]);
                    s = __ocml_add_rtn_f32(s, __ocml_mul_rtn_f32(a, fval(a > 0.0f ? d.x : d.y)));
                }
                const float num = __ocml_sub_rtp_f32(m.rhs[r], s);
                const float a = m.tcoef[t];
                const int x = m.tvar[t];
                const int2 dx = fdom(st, x);
                if (a > 0.0f) {
                    const int32_t k = fkey(canon_ub(div_ru(num, a)));
                    if (k < dx.y) {
                        __hip_atomic_fetch_min(&st[x].y, k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                        chg = true;
                        bad |= k < dx.x;
                    }
                } else {
                    const int32_t k = fkey(canon_lb(div_rd(num, a)));
                    if (k > dx.x) {
                        __hip_atomic_fetch_max(&st[x].x, k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                        chg = true;
                        bad |= k > dx.y;
                    }
                }
            }
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
    std::vector<int2> rowd(R);
    std::vector<int32_t> trow(T);
    for (int32_t r = 0; r < R; ++r) {
        const int32_t a0 = m->row_ptr[r], a1 = m->row_ptr[r + 1];
        if (!std::isfinite(m->rhs[r]))
            return internal_fail(PCCP_E_MODEL, "row " + std::to_string(r) + ": right-hand side must be finite");
        for (int32_t t = a0; t < a1; ++t) {
            const int32_t x = m->var[t];
            if (x < 0 || x >= V) return internal_fail(PCCP_E_MODEL, "row " + std::to_string(r) + ": variable out of range");
            if (!std::isfinite(m->coef[t]) || m->coef[t] == 0.0f)
                return internal_fail(PCCP_E_MODEL, "row " + std::to_string(r) + ": coefficient zero or not finite");
            if (seen[x]) return internal_fail(PCCP_E_MODEL, "row " + std::to_string(r) + ": variable repeated");
            seen[x] = 1;
            trow[t] = r;
        }
        for (int32_t t = a0; t < a1; ++t) seen[m->var[t]] = 0;
        rowd[r] = make_int2(a0, a1 - a0);
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
    const size_t o_tcoef = o_tvar + al(4 * (size_t)T), o_trow = o_tcoef + al(4 * (size_t)T);
    const size_t total = o_trow + al(4 * (size_t)T) + 256;
    std::vector<char> host(total, 0);
    if (R) {
        memcpy(host.data() + o_rowd, rowd.data(), 8 * (size_t)R);
        memcpy(host.data() + o_rhs, m->rhs.data(), 4 * (size_t)R);
    }
    if (T) {
        memcpy(host.data() + o_tvar, m->var.data(), 4 * (size_t)T);
        memcpy(host.data() + o_tcoef, m->coef.data(), 4 * (size_t)T);
        memcpy(host.data() + o_trow, trow.data(), 4 * (size_t)T);
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
    s->dev.trow = reinterpret_cast<const int32_t *>(base + o_trow);
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
