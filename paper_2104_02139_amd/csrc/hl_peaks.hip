// hl_peaks.hip -- what the device reaches on the two resources that bound
// the step kernels: a streaming copy (HBM read + write) and independent
// FP64 fused multiply-adds (the vector ALU).  The rooflines of the kernels
// are quoted against the vendor peaks; these two figures say how much of
// a vendor peak a plain kernel reaches on the same device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "hyperlag.h"

namespace {

// dst = src, grid-stride, U 16-byte loads in flight per lane
template <int U>
__global__ __launch_bounds__(256) void k_peak_copy(const double2 *__restrict__ src, double2 *__restrict__ dst,
                                                   int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i + (U - 1) * stride < n; i += U * stride) {
        double2 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = src[i + u * stride];
#pragma unroll
        for (int u = 0; u < U; ++u) dst[i + u * stride] = v[u];
    }
    for (; i < n; i += stride) dst[i] = src[i];
}

constexpr int kChains = 8;      // independent FMA chains per lane
constexpr int kFmaIter = 4096;  // FMAs per chain

// kChains independent chains of kFmaIter FMAs per lane; the sum is stored
// so that nothing is dropped.  flop per launch = 2 kChains kFmaIter lanes.
__global__ __launch_bounds__(256) void k_peak_fma(double *__restrict__ out, double b, double c) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double a[kChains];
#pragma unroll
    for (int j = 0; j < kChains; ++j) a[j] = 1.0 + 1e-3 * (double)((t + j) & 1023);
    for (int it = 0; it < kFmaIter; ++it) {
#pragma unroll
        for (int j = 0; j < kChains; ++j) a[j] = __fma_rn(a[j], b, c);
    }
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < kChains; ++j) s += a[j];
    out[t] = s;
}

struct Timer {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    bool ok = false;
    Timer() { ok = hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess; }
    ~Timer() {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    }
};

}  // namespace

extern "C" hl_status hl_measure_peaks(int device, void *hip_stream, int64_t copy_bytes, double *copy_gbs,
                                      double *fp64_tflops) {
    if (!copy_gbs || !fp64_tflops || copy_bytes < (1 << 20) || copy_bytes % 16 != 0) return HL_E_INVALID;
    if (hipSetDevice(device) != hipSuccess) return HL_E_HIP;
    hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
    const int64_t n2 = copy_bytes / 16;
    const unsigned fma_blocks = 256 * 16, copy_blocks = 1024;
    const int64_t fma_lanes = (int64_t)fma_blocks * 256;
    void *src = nullptr, *dst = nullptr, *out = nullptr;
    if (hipMalloc(&src, copy_bytes) != hipSuccess) return HL_E_OOM;
    if (hipMalloc(&dst, copy_bytes) != hipSuccess) {
        (void)hipFree(src);
        return HL_E_OOM;
    }
    if (hipMalloc(&out, sizeof(double) * fma_lanes) != hipSuccess) {
        (void)hipFree(src);
        (void)hipFree(dst);
        return HL_E_OOM;
    }
    hl_status st = HL_OK;
    {
        Timer tm;
        if (!tm.ok) st = HL_E_HIP;
        const auto *a = static_cast<const double2 *>(src);
        auto *b = static_cast<double2 *>(dst);
        float ms = 0.f;
        if (st == HL_OK && hipMemsetAsync(src, 0, copy_bytes, s) != hipSuccess) st = HL_E_HIP;
        // copy: the best of four launch shapes (1 or 4 loads in flight per
        // lane, 2048 or 8192 blocks), each 2 untimed launches and 10 timed
        *copy_gbs = 0.0;
        for (int shape = 0; shape < 4 && st == HL_OK; ++shape) {
            const unsigned nb = shape & 1 ? 8 * copy_blocks : 2 * copy_blocks;
            auto run = [&]() {
                if (shape < 2)
                    k_peak_copy<1><<<nb, 256, 0, s>>>(a, b, n2);
                else
                    k_peak_copy<4><<<nb, 256, 0, s>>>(a, b, n2);
            };
            for (int r = 0; r < 2; ++r) run();
            (void)hipEventRecord(tm.e0, s);
            for (int r = 0; r < 10; ++r) run();
            (void)hipEventRecord(tm.e1, s);
            if (hipEventSynchronize(tm.e1) != hipSuccess || hipEventElapsedTime(&ms, tm.e0, tm.e1) != hipSuccess ||
                !(ms > 0.f))
                st = HL_E_HIP;
            else
                *copy_gbs = std::max(*copy_gbs, 2.0 * (double)copy_bytes * 10.0 / (1e-3 * ms) / 1e9);
        }
        if (st == HL_OK) {
            // FMA: 1 untimed launch, then 5 timed ones
            double *o = static_cast<double *>(out);
            k_peak_fma<<<fma_blocks, 256, 0, s>>>(o, 1.0000001, 1e-9);
            (void)hipEventRecord(tm.e0, s);
            for (int r = 0; r < 5; ++r) k_peak_fma<<<fma_blocks, 256, 0, s>>>(o, 1.0000001, 1e-9);
            (void)hipEventRecord(tm.e1, s);
            if (hipEventSynchronize(tm.e1) != hipSuccess || hipEventElapsedTime(&ms, tm.e0, tm.e1) != hipSuccess ||
                !(ms > 0.f))
                st = HL_E_HIP;
            else
                *fp64_tflops = 2.0 * kChains * (double)kFmaIter * (double)fma_lanes * 5.0 / (1e-3 * ms) / 1e12;
        }
        if (st == HL_OK && hipGetLastError() != hipSuccess) st = HL_E_HIP;
    }
    (void)hipStreamSynchronize(s);
    (void)hipFree(src);
    (void)hipFree(dst);
    (void)hipFree(out);
    return st;
}
