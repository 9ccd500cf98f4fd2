// Microbenchmarks of the device's attainable matrix-core rate and HBM copy
// bandwidth, the ceilings the roofline of the sigma kernels is read against.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "../../include/lrcc.h"
#include "common.hpp"

namespace lrcc {

namespace {
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

// every wave runs iters x kChains 16x16x4 products on kChains independent accumulators;
// one value per thread is written so that nothing is optimised away
template <typename T, int kChains>
__global__ void __launch_bounds__(kPeakThreads) k_mfma_peak(T *out, int iters, T seed) {
    typedef typename PeakMfma<T>::v4 v4;
    v4 acc[kChains];
#pragma unroll
    for (int j = 0; j < kChains; ++j) acc[j] = v4{0, 0, 0, 0};
    const T a = seed + (T)(threadIdx.x & 63) * (T)1e-3, b = seed - (T)(threadIdx.x >> 6) * (T)1e-3;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int j = 0; j < kChains; ++j) acc[j] = PeakMfma<T>::mma(a, b, acc[j]);
    }
    T s = 0;
#pragma unroll
    for (int j = 0; j < kChains; ++j) s += acc[j][0] + acc[j][1] + acc[j][2] + acc[j][3];
    out[blockIdx.x * kPeakThreads + threadIdx.x] = s;
}

// streaming copy with 16-byte accesses, four in flight per thread, grid-stride over
// groups of 4 * blockDim consecutive vectors (n a multiple of 4 * blockDim)
__global__ void __launch_bounds__(kPeakThreads) k_copy16(const float4 *in, float4 *out, i64 n) {
    const i64 step = (i64)gridDim.x * blockDim.x * 4;
    for (i64 t = blockIdx.x * (i64)blockDim.x * 4 + threadIdx.x; t < n; t += step) {
        float4 v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = in[t + u * blockDim.x];
#pragma unroll
        for (int u = 0; u < 4; ++u) out[t + u * blockDim.x] = v[u];
    }
}

template <typename T, int kChains>
double mfma_rate(int blocks, int iters, T *buf) {
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return -1;
    hipLaunchKernelGGL((k_mfma_peak<T, kChains>), dim3(blocks), dim3(kPeakThreads), 0, 0, buf, iters / 4, (T)1);
    (void)hipEventRecord(e0, 0);
    hipLaunchKernelGGL((k_mfma_peak<T, kChains>), dim3(blocks), dim3(kPeakThreads), 0, 0, buf, iters, (T)1);
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
    // best over 1, 2 and 4 waves per SIMD (4, 8, 16 workgroups of four waves per compute
    // unit) and 8 or 16 independent accumulators per wave
    const int cus = std::max(1, prop.multiProcessorCount);
    void *buf = nullptr;
    if (hipMalloc(&buf, (size_t)cus * 16 * kPeakThreads * sizeof(double)) != hipSuccess) return LRCC_E_OOM;
    double f32 = -1, f64 = -1;
    for (int wps : {1, 2, 4}) {
        const int blocks = cus * 4 * wps;
        f32 = std::max({f32, mfma_rate<float, 8>(blocks, 20000 / wps, (float *)buf),
                        mfma_rate<float, 16>(blocks, 10000 / wps, (float *)buf)});
        f64 = std::max({f64, mfma_rate<double, 8>(blocks, 10000 / wps, (double *)buf),
                        mfma_rate<double, 16>(blocks, 5000 / wps, (double *)buf)});
    }
    (void)hipFree(buf);
    *mfma_f32_tflops = f32;
    *mfma_f64_tflops = f64;
    if (f32 <= 0 || f64 <= 0) return LRCC_E_HIP;
    // HBM: copy of 2 GiB (2 GiB read + 2 GiB written) per launch, the first run of each grid
    // size a warm-up
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
    for (int rep = 0; rep < 6; ++rep) {
        const int grid = cus * (rep < 3 ? 16 : 64);
        (void)hipEventRecord(e0, 0);
        hipLaunchKernelGGL(k_copy16, dim3(grid), dim3(kPeakThreads), 0, 0, (const float4 *)a, (float4 *)b, n);
        (void)hipEventRecord(e1, 0);
        if (hipEventSynchronize(e1) != hipSuccess) break;
        float ms = 0;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (rep != 0 && rep != 3) best = std::max(best, 2.0 * bytes / (ms * 1e-3) / 1e9);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(a);
    (void)hipFree(b);
    *hbm_copy_gbs = best;
    return hipGetLastError() == hipSuccess && best > 0 ? LRCC_OK : LRCC_E_HIP;
}
