// LDS peaks of the device (the denominators of the propagation loop's
// roofline): 64-bit LDS reads, and 32-bit LDS atomic max with and without
// the old value returned, each over every compute unit with a
// conflict-free pattern (the 64 lanes of a wavefront touch 64 consecutive
// words).  Every kernel keeps its results live through one global store per
// thread so that no access is removed.
#include <hip/hip_runtime.h>

#include <string>

#include "../../include/pccp.h"
#include "pccp_launch.h"

namespace pccp {
namespace {

constexpr int kMicroBlock = 256;
constexpr int kMicroWords = 8192;       // 32 KiB of LDS per workgroup (int32 words)
constexpr int kMicroIters = 2048;
constexpr int kMicroUnroll = 8;

// each thread reads int2 pairs tid + k * stride (mod the array), 8
// independent loads in flight per step.  The stride and the stored values
// come from the host at run time and every value enters a running
// multiply-add, so the compiler can neither see that the addresses repeat
// nor fold the loop into a closed form: every load is issued.
__global__ __launch_bounds__(kMicroBlock) void lds_read_kernel(int *sink, int stride, int seed)
{
    __shared__ int2 a[kMicroWords / 2];
    const int tid = threadIdx.x;
    for (int i = tid; i < kMicroWords / 2; i += kMicroBlock) a[i] = make_int2(i ^ seed, ~i + seed);
    __syncthreads();
    int acc0 = 0, acc1 = 0;
    constexpr int N = kMicroWords / 2;
    for (int it = 0; it < kMicroIters; ++it) {
        int2 v[kMicroUnroll];
#pragma unroll
        for (int u = 0; u < kMicroUnroll; ++u)
            v[u] = a[(tid + (it * kMicroUnroll + u) * stride) & (N - 1)];
#pragma unroll
        for (int u = 0; u < kMicroUnroll; ++u) {
            acc0 = acc0 * 3 + v[u].x;
            acc1 ^= v[u].y;
        }
    }
    sink[blockIdx.x * kMicroBlock + tid] = acc0 ^ acc1;
}

// each lane joins a rising value into word lane + 64 k of its wavefront's
// region: every operation is a real read-modify-write
template <bool RET>
__global__ __launch_bounds__(kMicroBlock) void lds_atomic_kernel(int *sink)
{
    __shared__ int a[kMicroWords];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    for (int i = tid; i < kMicroWords; i += kMicroBlock) a[i] = 0;
    __syncthreads();
    constexpr int R = kMicroWords / (kMicroBlock / 64);   // words per wavefront
    int *w = a + wid * R;
    int acc = 0;
    for (int it = 0; it < kMicroIters; ++it) {
#pragma unroll
        for (int u = 0; u < kMicroUnroll; ++u) {
            int *p = w + ((lane + 64 * (it * kMicroUnroll + u)) & (R - 1));
            const int v = it * kMicroUnroll + u + 1;
            if (RET)
                acc += __hip_atomic_fetch_max(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            else
                __hip_atomic_fetch_max(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
    }
    __syncthreads();
    sink[blockIdx.x * kMicroBlock + tid] = acc + a[tid];
}

}  // namespace
}  // namespace pccp

using namespace pccp;

extern "C" int32_t pccp_measure_lds_peaks(pccp_lds_peaks *out)
{
    if (!out) return internal_fail(PCCP_E_INVALID_ARG, "pccp_measure_lds_peaks: out is NULL");
    *out = pccp_lds_peaks{};
    int dev = 0;
    hipDeviceProp_t prop;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipGetDeviceProperties(&prop, dev);
    if (e != hipSuccess)
        return internal_fail(PCCP_E_DEVICE, std::string("device query: ") + hipGetErrorString(e));
    // 8 workgroups of 256 threads per compute unit: 32 KiB of LDS each fits,
    // and 8 wavefronts per SIMD keep the LDS pipeline busy
    const int grid = prop.multiProcessorCount * 8;
    int *sink = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    e = hipMalloc(&sink, sizeof(int) * (size_t)grid * kMicroBlock);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    float ms[3] = {0, 0, 0};
    for (int k = 0; k < 3 && e == hipSuccess; ++k) {
        for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) {   // the first run warms up
            e = hipEventRecord(e0, 0);
            // stride 256: the 64 lanes of a wavefront read 64 consecutive
            // pairs (512 bytes), conflict-free
            if (k == 0) hipLaunchKernelGGL(lds_read_kernel, dim3(grid), dim3(kMicroBlock), 0, 0, sink,
                                           kMicroBlock, 0x5bd1e995);
            if (k == 1) hipLaunchKernelGGL(lds_atomic_kernel<false>, dim3(grid), dim3(kMicroBlock), 0, 0, sink);
            if (k == 2) hipLaunchKernelGGL(lds_atomic_kernel<true>, dim3(grid), dim3(kMicroBlock), 0, 0, sink);
            if (e == hipSuccess) e = hipGetLastError();
            if (e == hipSuccess) e = hipEventRecord(e1, 0);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            if (e == hipSuccess) e = hipEventElapsedTime(&ms[k], e0, e1);
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (sink) (void)hipFree(sink);
    if (e != hipSuccess)
        return internal_fail(PCCP_E_DEVICE, std::string("LDS peaks: ") + hipGetErrorString(e));
    const double ops = (double)grid * kMicroBlock * kMicroIters * kMicroUnroll;
    out->read_gbs = ops * 8.0 / (ms[0] * 1e-3) / 1e9;
    out->atomic_gops = ops / (ms[1] * 1e-3) / 1e9;
    out->atomic_ret_gops = ops / (ms[2] * 1e-3) / 1e9;
    for (int k = 0; k < 3; ++k) out->ms[k] = ms[k];
    out->num_cus = prop.multiProcessorCount;
    out->grid = grid;
    out->block = kMicroBlock;
    return PCCP_OK;
}
