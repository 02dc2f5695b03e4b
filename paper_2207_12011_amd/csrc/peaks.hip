// peaks.hip -- measured ceilings of the device, against which the renderer's rates are quoted.
//
// The ray march is bound by FP32 vector arithmetic and its data moves through HBM; the vendor's peak
// figures for both are theoretical, so the library measures what a simple kernel reaches on the
// device at hand:
//  * copy bandwidth: a STREAM-like copy of a 1 GiB float32 array into another (16-byte loads and
//    stores, grid-stride), counted as 2 GiB moved per pass;
//  * FP32 fused multiply-add rate: every lane runs eight independent chains of dependent FMAs
//    (built without packed FP32, so one FMA is one lane operation per cycle), in enough waves to
//    fill every SIMD; counted as lane operations per second (one FMA = one operation, the unit the
//    renderer's arithmetic is counted in).
// Each is timed with HIP events over several passes after a warm-up pass, and the best pass is kept.
#include <algorithm>

#include "internal.h"

namespace raypc {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));

// Each thread moves four 16-byte elements per round, all four loads issued before the stores;
// n is a multiple of 4 x the grid's thread count (the host sizes it so).
__global__ __launch_bounds__(256) void copy_kernel(const f32x4* __restrict__ src, f32x4* __restrict__ dst, size_t n) {
    const size_t stride = static_cast<size_t>(gridDim.x) * blockDim.x;
    for (size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += 4 * stride) {
        const f32x4 a = __builtin_nontemporal_load(src + i), b = __builtin_nontemporal_load(src + i + stride);
        const f32x4 c = __builtin_nontemporal_load(src + i + 2 * stride), d = __builtin_nontemporal_load(src + i + 3 * stride);
        __builtin_nontemporal_store(a, dst + i);
        __builtin_nontemporal_store(b, dst + i + stride);
        __builtin_nontemporal_store(c, dst + i + 2 * stride);
        __builtin_nontemporal_store(d, dst + i + 3 * stride);
    }
}

constexpr int kChains = 8;
constexpr int kFmaIters = 4096;

__global__ __launch_bounds__(256) void fma_kernel(float a, float b, float* out) {
    float v[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) v[c] = static_cast<float>(threadIdx.x + c);
    for (int i = 0; i < kFmaIters; ++i) {
#pragma unroll
        for (int c = 0; c < kChains; ++c) v[c] = fmaf(v[c], a, b);
    }
    float s = 0.0f;
#pragma unroll
    for (int c = 0; c < kChains; ++c) s += v[c];
    // never true for the arguments the host passes (a = 1, b = 0): keeps the chains live
    if (s == -1.0f) out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

}  // namespace

hipError_t measure_peaks(double* copy_bytes_per_s, double* fma_ops_per_s, hipStream_t s) {
    const size_t bytes = size_t(1) << 30;
    const size_t n4 = bytes / sizeof(f32x4);
    f32x4 *src = nullptr, *dst = nullptr;
    float* sink = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipMalloc(reinterpret_cast<void**>(&src), bytes);
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&dst), bytes);
    int cus = 0;
    if (e == hipSuccess) {
        int dev = 0;
        e = hipGetDevice(&dev);
        if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    }
    // 8 waves on each of the 4 SIMDs of every CU, several rounds over the device
    const unsigned fma_blocks = static_cast<unsigned>(std::max(cus, 1)) * 8u * 4u;
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&sink), size_t(fma_blocks) * 256 * sizeof(float));
    if (e == hipSuccess) e = hipMemsetAsync(src, 0, bytes, s);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    double best_copy = 0.0, best_fma = 0.0;
    // a power-of-two grid that divides the 2^26 elements into whole rounds of four
    const unsigned copy_blocks = 4096u;
    for (int pass = 0; e == hipSuccess && pass < 6; ++pass) {
        e = hipEventRecord(e0, s);
        if (e == hipSuccess) {
            hipLaunchKernelGGL(copy_kernel, dim3(copy_blocks), dim3(256), 0, s, src, dst, n4);
            e = hipGetLastError();
        }
        if (e == hipSuccess) e = hipEventRecord(e1, s);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e == hipSuccess && pass > 0 && ms > 0.0f) best_copy = std::max(best_copy, 2.0 * bytes / (ms * 1e-3));
    }
    for (int pass = 0; e == hipSuccess && pass < 6; ++pass) {
        e = hipEventRecord(e0, s);
        if (e == hipSuccess) {
            hipLaunchKernelGGL(fma_kernel, dim3(fma_blocks), dim3(256), 0, s, 1.0f, 0.0f, sink);
            e = hipGetLastError();
        }
        if (e == hipSuccess) e = hipEventRecord(e1, s);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        const double ops = double(fma_blocks) * 256.0 * kFmaIters * kChains;
        if (e == hipSuccess && pass > 0 && ms > 0.0f) best_fma = std::max(best_fma, ops / (ms * 1e-3));
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(src);
    (void)hipFree(dst);
    (void)hipFree(sink);
    *copy_bytes_per_s = best_copy;
    *fma_ops_per_s = best_fma;
    return e;
}

}  // namespace raypc
