// Achievable peaks of the device, for roofline reports: a plain stream copy
// (HBM bandwidth) and a loop of independent FP32 fused multiply-adds (VALU
// rate), each timed with HIP events on the caller's stream.
#include <cstdio>
#include <string>

#include "vd.h"
#include "vd_internal.h"

namespace vd {
namespace {

__global__ __launch_bounds__(256) void k_copy(const float4* __restrict__ src, float4* __restrict__ dst, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

// Eight independent FMA chains per lane (enough to cover the FMA latency);
// the results are stored so that nothing is optimised away.
constexpr int kFmaChains = 8;
__global__ __launch_bounds__(256) void k_fma(float* out, int iters, float b, float c) {
    float a[kFmaChains];
#pragma unroll
    for (int k = 0; k < kFmaChains; ++k) a[k] = (float)(threadIdx.x + k);
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int k = 0; k < kFmaChains; ++k) a[k] = fmaf(a[k], b, c);
    }
    float s = 0.f;
#pragma unroll
    for (int k = 0; k < kFmaChains; ++k) s += a[k];
    out[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

}  // namespace
}  // namespace vd

extern "C" {

VD_API vd_status vd_measure_peaks(int device, void* stream, double* copy_gbs, double* fma_tops) {
    if (!copy_gbs || !fma_tops) return VD_ERR_INVALID_ARG;
    if (hipSetDevice(device) != hipSuccess) return VD_ERR_HIP;
    hipStream_t s = static_cast<hipStream_t>(stream);
    int num_cu = 256;
    if (hipDeviceGetAttribute(&num_cu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) num_cu = 256;
    const int64_t n4 = (int64_t)1 << 26;  // 1 GiB of float4 per buffer
    float4 *a = nullptr, *b = nullptr;
    float* out = nullptr;
    const int fma_blocks = num_cu * 16;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    vd_status st = VD_OK;
    if (hipMalloc(&a, n4 * sizeof(float4)) != hipSuccess || hipMalloc(&b, n4 * sizeof(float4)) != hipSuccess ||
        hipMalloc(&out, (size_t)fma_blocks * 256 * sizeof(float)) != hipSuccess) {
        st = VD_ERR_OOM;
    } else if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess ||
               hipMemsetAsync(a, 0, n4 * sizeof(float4), s) != hipSuccess) {
        st = VD_ERR_HIP;
    } else {
        // best of five runs each
        float best_copy = 1e30f, best_fma = 1e30f;
        const int iters = 1 << 15;
        for (int r = 0; r < 6 && st == VD_OK; ++r) {
            float ms = 0.f;
            if (hipEventRecord(e0, s) != hipSuccess) st = VD_ERR_HIP;
            hipLaunchKernelGGL(vd::k_copy, dim3(num_cu * 8), dim3(256), 0, s, a, b, n4);
            if (hipGetLastError() != hipSuccess || hipEventRecord(e1, s) != hipSuccess ||
                hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
                st = VD_ERR_HIP;
            if (r > 0 && ms < best_copy) best_copy = ms;
            if (hipEventRecord(e0, s) != hipSuccess) st = VD_ERR_HIP;
            hipLaunchKernelGGL(vd::k_fma, dim3(fma_blocks), dim3(256), 0, s, out, iters, 0.999f, 1e-3f);
            if (hipGetLastError() != hipSuccess || hipEventRecord(e1, s) != hipSuccess ||
                hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
                st = VD_ERR_HIP;
            if (r > 0 && ms < best_fma) best_fma = ms;
        }
        if (st == VD_OK) {
            *copy_gbs = 2.0 * (double)n4 * sizeof(float4) / (best_copy * 1e-3) / 1e9;
            *fma_tops = (double)fma_blocks * 256.0 * iters * vd::kFmaChains / (best_fma * 1e-3) / 1e12;
        }
    }
    // release what was taken; a failure here cannot change the result
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (a) (void)hipFree(a);
    if (b) (void)hipFree(b);
    if (out) (void)hipFree(out);
    return st;
}

}  // extern "C"
