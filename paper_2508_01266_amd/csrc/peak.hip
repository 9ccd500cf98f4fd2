// Microbenchmarks of the device's attainable matrix-core rate and HBM copy
// bandwidth, the ceilings the roofline of the sigma kernels is read against.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "../../include/lrcc.h"
#include "common.hpp"

namespace lrcc {

namespace {
constexpr int kChains = 8;       // independent accumulators per wave (hides the MFMA latency)
constexpr int kPeakThreads = 256;

template <typename T> struct PeakMfma;
template <> struct PeakMfma<float> {
    typedef float v4 __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ v4 mma(float a, float b, v4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
};
template <> struct PeakMfma<double> {
    typedef double v4 __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ v4 mma(double a, double b, v4 c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
};

// every wave runs iters x kChains dependent-free 16x16x4 products; one value per thread
// is written so that nothing is optimised away
template <typename T>
__global__ void __launch_bounds__(kPeakThreads) k_mfma_peak(T *out, int iters, T seed) {
    typedef typename PeakMfma<T>::v4 v4;
    v4 acc[kChains];
#pragma unroll
    for (int j = 0; j < kChains; ++j) acc[j] = v4{0, 0, 0, 0};
    T a = seed + (T)(threadIdx.x & 63) * (T)1e-3, b = seed - (T)(threadIdx.x >> 6) * (T)1e-3;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int j = 0; j < kChains; ++j) acc[j] = PeakMfma<T>::mma(a, b, acc[j]);
        a = a * (T)0.999999;
    }
    T s = 0;
#pragma unroll
    for (int j = 0; j < kChains; ++j) s += acc[j][0] + acc[j][1] + acc[j][2] + acc[j][3];
    out[blockIdx.x * kPeakThreads + threadIdx.x] = s;
}

// streaming copy with 16-byte accesses, grid-stride
__global__ void __launch_bounds__(kPeakThreads) k_copy16(const float4 *in, float4 *out, i64 n) {
    for (i64 t = blockIdx.x * (i64)blockDim.x + threadIdx.x; t < n; t += (i64)gridDim.x * blockDim.x) out[t] = in[t];
}

template <typename T>
double mfma_rate(int blocks, int iters, T *buf) {
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return -1;
    hipLaunchKernelGGL(k_mfma_peak<T>, dim3(blocks), dim3(kPeakThreads), 0, 0, buf, iters / 4, (T)1);
    (void)hipEventRecord(e0, 0);
    hipLaunchKernelGGL(k_mfma_peak<T>, dim3(blocks), dim3(kPeakThreads), 0, 0, buf, iters, (T)1);
    (void)hipEventRecord(e1, 0);
    double r = -1;
    if (hipEventSynchronize(e1) == hipSuccess && hipGetLastError() == hipSuccess) {
        float ms = 0;
        (void)hipEventElapsedTime(&ms, e0, e1);
        const double flops = (double)blocks * (kPeakThreads / 64) * iters * kChains * (16.0 * 16 * 4 * 2);
        r = flops / (ms * 1e-3) / 1e12;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return r;
}
}  // namespace

}  // namespace lrcc

using namespace lrcc;

extern "C" lrcc_status lrcc_measure_peaks(int hip_device, double *mfma_f32_tflops, double *mfma_f64_tflops,
                                          double *hbm_copy_gbs) {
    if (!mfma_f32_tflops || !mfma_f64_tflops || !hbm_copy_gbs) return LRCC_E_ARG;
    if (hipSetDevice(hip_device) != hipSuccess) return LRCC_E_HIP;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, hip_device) != hipSuccess) return LRCC_E_HIP;
    // eight workgroups of four waves per compute unit: two waves per SIMD, as the ladder runs
    const int blocks = std::max(1, prop.multiProcessorCount) * 8;
    void *buf = nullptr;
    if (hipMalloc(&buf, (size_t)blocks * kPeakThreads * sizeof(double)) != hipSuccess) return LRCC_E_OOM;
    *mfma_f32_tflops = mfma_rate<float>(blocks, 20000, (float *)buf);
    *mfma_f64_tflops = mfma_rate<double>(blocks, 10000, (double *)buf);
    (void)hipFree(buf);
    if (*mfma_f32_tflops < 0 || *mfma_f64_tflops < 0) return LRCC_E_HIP;
    // HBM: copy of 2 GiB (2 GiB read + 2 GiB written) per launch, best of three
    const size_t bytes = (size_t)2 << 30;
    void *a = nullptr, *b = nullptr;
    if (hipMalloc(&a, bytes) != hipSuccess) return LRCC_E_OOM;
    if (hipMalloc(&b, bytes) != hipSuccess) { (void)hipFree(a); return LRCC_E_OOM; }
    (void)hipMemset(a, 0, bytes);
    const i64 n = (i64)(bytes / 16);
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    double best = 0;
    const int grid = std::max(1, prop.multiProcessorCount) * 16;
    for (int rep = 0; rep < 4; ++rep) {
        (void)hipEventRecord(e0, 0);
        hipLaunchKernelGGL(k_copy16, dim3(grid), dim3(kPeakThreads), 0, 0, (const float4 *)a, (float4 *)b, n);
        (void)hipEventRecord(e1, 0);
        if (hipEventSynchronize(e1) != hipSuccess) break;
        float ms = 0;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (rep > 0) best = std::max(best, 2.0 * bytes / (ms * 1e-3) / 1e9);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(a);
    (void)hipFree(b);
    *hbm_copy_gbs = best;
    return hipGetLastError() == hipSuccess && best > 0 ? LRCC_OK : LRCC_E_HIP;
}
