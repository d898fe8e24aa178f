// Measured ceilings of the device, the denominators beside the datasheet
// peaks in the roofline fractions: a streaming copy (HBM bandwidth), a loop
// of independent FP64 fused multiply-adds (vector FP64 rate) and a loop of
// FP64 matrix-core products (v_mfma_f64_16x16x4).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "../../include/iga_trim.h"
#include "common.hpp"

namespace iga {

// dst = src, 16 bytes per load and store, grid-stride.
__global__ void __launch_bounds__(256) k_peak_copy(const double2* __restrict__ src, double2* __restrict__ dst,
                                                   int64_t n2) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n2; i += stride) dst[i] = src[i];
}

// kChains independent chains of a = a * b + c per thread, iters rounds; the
// sum is stored so the loop is not removed.
constexpr int kChains = 16;
__global__ void __launch_bounds__(256) k_peak_fma(double* __restrict__ out, int iters, double b, double c) {
    double a[kChains];
#pragma unroll
    for (int k = 0; k < kChains; ++k) a[k] = (double)(threadIdx.x + k);
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int k = 0; k < kChains; ++k) a[k] = fma(a[k], b, c);
    }
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < kChains; ++k) s += a[k];
    out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

typedef double peak_f64x4 __attribute__((ext_vector_type(4)));
constexpr int kMfmaChains = 4;
// kMfmaChains independent accumulators per wavefront, iters rounds of
// 16x16x4 FP64 products (2 * 16 * 16 * 4 flops each).
__global__ void __launch_bounds__(256) k_peak_mfma(double* __restrict__ out, int iters, double x) {
    peak_f64x4 acc[kMfmaChains];
#pragma unroll
    for (int k = 0; k < kMfmaChains; ++k) acc[k] = peak_f64x4{0.0, 0.0, 0.0, 0.0};
    const double a = x + threadIdx.x * 1e-3, b = x - threadIdx.x * 1e-3;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int k = 0; k < kMfmaChains; ++k) acc[k] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[k], 0, 0, 0);
    }
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < kMfmaChains; ++k) s += acc[k][0] + acc[k][1] + acc[k][2] + acc[k][3];
    out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

}  // namespace iga

using namespace iga;

extern "C" {

int iga_measure_peaks(const double* src, double* dst, int64_t n, int32_t reps, iga_peaks* out, void* stream) {
    try {
        IGA_REQUIRE(src && dst && out && n >= 2 && reps > 0, IGA_E_INVALID, "bad calibration arguments");
        hipStream_t s = (hipStream_t)stream;
        int dev = 0, n_cu = 0;
        HIPX(hipGetDevice(&dev));
        HIPX(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev));
        hipEvent_t a, b;
        HIPX(hipEventCreate(&a));
        HIPX(hipEventCreate(&b));
        auto timed = [&](auto launch) {
            launch();  // warm-up
            float best = 1e30f;
            for (int r = 0; r < reps; ++r) {
                HIPX(hipEventRecord(a, s));
                launch();
                HIPX(hipEventRecord(b, s));
                HIPX(hipEventSynchronize(b));
                float ms = 0.f;
                HIPX(hipEventElapsedTime(&ms, a, b));
                best = std::min(best, ms);
            }
            return (double)best;
        };
        const int64_t n2 = n / 2;
        const int copy_blocks = n_cu * 16;
        double ms = timed([&] {
            hipLaunchKernelGGL(k_peak_copy, dim3(copy_blocks), dim3(256), 0, s, reinterpret_cast<const double2*>(src),
                               reinterpret_cast<double2*>(dst), n2);
        });
        out->copy_gbs = 2.0 * 16.0 * (double)n2 / (ms * 1e-3) / 1e9;
        // FMA loop: 8 workgroups per CU (8 waves per SIMD pair), 2 flops per FMA
        const int fma_blocks = n_cu * 8, fma_iters = 4096;
        IGA_REQUIRE((int64_t)fma_blocks * 256 <= n, IGA_E_INVALID, "calibration buffer too small");
        ms = timed([&] { hipLaunchKernelGGL(k_peak_fma, dim3(fma_blocks), dim3(256), 0, s, dst, fma_iters, 0.999, 1e-3); });
        out->fma_tflops = 2.0 * kChains * (double)fma_iters * fma_blocks * 256 / (ms * 1e-3) / 1e12;
        const int mfma_iters = 4096;
        ms = timed([&] { hipLaunchKernelGGL(k_peak_mfma, dim3(fma_blocks), dim3(256), 0, s, dst, mfma_iters, 0.5); });
        const double waves = (double)fma_blocks * 4;
        out->mfma_f64_tflops = 2.0 * 16 * 16 * 4 * kMfmaChains * (double)mfma_iters * waves / (ms * 1e-3) / 1e12;
        out->n_cu = n_cu;
        hipEventDestroy(a);
        hipEventDestroy(b);
        HIPX(hipGetLastError());
    } catch (const Error& e) {
        set_error(e.msg);
        return e.code;
    }
    return IGA_OK;
}

}  // extern "C"
