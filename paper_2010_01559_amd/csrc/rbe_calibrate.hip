// rbe_calibrate.hip -- throughput micro-benchmarks of the device: the
// hardware sine/cosine of revolutions, FP32 and FP64 fused multiply-adds,
// and a device copy.  They calibrate the rooflines the benchmark reports
// for the kernels (operation counts per particle-mode pair in the paper's
// cost model, Sec. 3.1).  Built with the library's own flags, so the FP32
// figure is that of non-packed instructions, the ones the kernels issue.
//
// Each arithmetic kernel runs 16 independent dependency chains per lane
// (enough to hide the pipeline latency with 8 waves per SIMD) for `iters`
// rounds; the lane results are folded into one store that a never-true
// test guards, so the work cannot be dropped.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include <algorithm>

#include "rbe_internal.h"

namespace rbe {

constexpr int kCalChains = 16;
constexpr int kCalBlock = 256;

__global__ __launch_bounds__(kCalBlock) void k_cal_trans(float *out, int iters, float seed)
{
    float x[kCalChains];
#pragma unroll
    for (int k = 0; k < kCalChains; ++k) x[k] = seed + 1e-3f * (float)(threadIdx.x + 7 * k);
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int k = 0; k < kCalChains; ++k)
            x[k] = (k & 1) ? __builtin_amdgcn_cosf(x[k]) : __builtin_amdgcn_sinf(x[k]);
    }
    float s = 0.0f;
#pragma unroll
    for (int k = 0; k < kCalChains; ++k) s += x[k];
    if (s == 1234.5f) out[blockIdx.x] = s;
}

template <typename T>
__global__ __launch_bounds__(kCalBlock) void k_cal_fma(T *out, int iters, T seed)
{
    T x[kCalChains];
    const T a = (T)0.999, b = (T)1e-3;
#pragma unroll
    for (int k = 0; k < kCalChains; ++k) x[k] = seed + (T)1e-3 * (T)(threadIdx.x + 7 * k);
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int k = 0; k < kCalChains; ++k) x[k] = fma(x[k], a, b);
    }
    T s = 0;
#pragma unroll
    for (int k = 0; k < kCalChains; ++k) s += x[k];
    if (s == (T)1234.5) out[blockIdx.x] = s;
}

__global__ __launch_bounds__(kCalBlock) void k_cal_copy(const float4 *__restrict__ src, float4 *__restrict__ dst,
                                                        int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * kCalBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kCalBlock)
        dst[i] = src[i];
}

}  // namespace rbe

using namespace rbe;

extern "C" rbe_status rbe_calibrate(int32_t kind, int32_t reps, double *rate)
{
    if (!rate || kind < 0 || kind > 3) return RBE_ERR_INVALID;
    if (reps < 1) reps = 1;
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
        (void)hipGetLastError();
        return RBE_ERR_NO_DEVICE;
    }
    const int blocks = prop.multiProcessorCount * 8;   // 32 waves per compute unit
    const int iters = 4096;
    const int64_t copy_n = (int64_t)(256u << 20) / (int64_t)sizeof(float4);
    void *buf = nullptr, *buf2 = nullptr;
    const size_t bytes = kind == 3 ? (size_t)copy_n * sizeof(float4) : sizeof(double) * blocks;
    if (hipMalloc(&buf, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return RBE_ERR_OOM;
    }
    if (kind == 3 && hipMalloc(&buf2, bytes) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipFree(buf);
        return RBE_ERR_OOM;
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    rbe_status st = RBE_OK;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) st = RBE_ERR_HIP;
    auto launch = [&]() {
        switch (kind) {
        case 0:
            launch_k(k_cal_trans, blocks, kCalBlock, 0, nullptr, (float *)buf, iters, 0.123f);
            break;
        case 1:
            launch_k(k_cal_fma<float>, blocks, kCalBlock, 0, nullptr, (float *)buf, iters, 0.123f);
            break;
        case 2:
            launch_k(k_cal_fma<double>, blocks, kCalBlock, 0, nullptr, (double *)buf, iters, 0.123);
            break;
        default:
            launch_k(k_cal_copy, prop.multiProcessorCount * 16, kCalBlock, 0, nullptr, (const float4 *)buf,
                     (float4 *)buf2, copy_n);
            break;
        }
    };
    double best = 0.0;
    if (st == RBE_OK) {
        launch();   // warm-up
        for (int r = 0; r < reps && st == RBE_OK; ++r) {
            float ms = 0.0f;
            if (hipEventRecord(e0, nullptr) != hipSuccess) st = RBE_ERR_HIP;
            launch();
            if (st == RBE_OK && (hipEventRecord(e1, nullptr) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                                 hipEventElapsedTime(&ms, e0, e1) != hipSuccess || hipGetLastError() != hipSuccess))
                st = RBE_ERR_HIP;
            const double work = kind == 3 ? 2.0 * (double)bytes
                                          : (double)blocks * kCalBlock * (double)iters * (double)kCalChains;
            if (st == RBE_OK && ms > 0.0f) best = std::max(best, work / (1e-3 * (double)ms));
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(buf);
    if (buf2) (void)hipFree(buf2);
    *rate = best;
    return st;
}
