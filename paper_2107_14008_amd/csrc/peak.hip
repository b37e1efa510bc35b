// Measured vector-ALU peak of the device: the denominator against which the
// pair kernels' flop rates are read beside the published figures.  Every
// lane runs kChains independent chains of fused multiply-adds
// (v = v a + b), enough independent work to hide the FMA latency, on
// kWgPerCu workgroups of 256 lanes per CU, timed with HIP events around the
// launch.  float32 is built like every kernel here, without packed FP32
// instructions, so this is the rate the float32 pair kernels can reach.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>

#include "pmfmm_peak.h"

namespace {

constexpr int kChains = 8;
constexpr int kUnroll = 8;
constexpr int kWgPerCu = 8;
constexpr int kLanes = 256;

template <class T>
__global__ void __launch_bounds__(kLanes) fma_chains(T* __restrict__ out, int32_t iters, T a, T b) {
    T v[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) v[c] = (T)(threadIdx.x & 7) + (T)c;
    for (int32_t i = 0; i < iters; ++i) {
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
#pragma unroll
            for (int c = 0; c < kChains; ++c) v[c] = fma(v[c], a, b);
        }
    }
    T s = 0;
#pragma unroll
    for (int c = 0; c < kChains; ++c) s += v[c];
    out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

thread_local std::string g_peak_err;

template <class T>
int run(int32_t iters, double* tflops, double* ms_out) {
    int dev = 0, n_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
        g_peak_err = "no HIP device";
        return PMFMM_PEAK_EDEVICE;
    }
    const int grid = n_cu * kWgPerCu;
    T* out = nullptr;
    if (hipMalloc(&out, (size_t)grid * kLanes * sizeof(T)) != hipSuccess) {
        g_peak_err = "hipMalloc failed";
        return PMFMM_PEAK_EDEVICE;
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = PMFMM_PEAK_EDEVICE;
    float ms = 0.f;
    // a and b keep the chains bounded and are not compile-time constants
    const T a = (T)0.999999, b = (T)1e-3;
    if (hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess) {
        hipLaunchKernelGGL(fma_chains<T>, dim3(grid), dim3(kLanes), 0, nullptr, out, iters / 16, a, b);
        if (hipEventRecord(e0, nullptr) == hipSuccess) {
            hipLaunchKernelGGL(fma_chains<T>, dim3(grid), dim3(kLanes), 0, nullptr, out, iters, a, b);
            if (hipGetLastError() == hipSuccess && hipEventRecord(e1, nullptr) == hipSuccess &&
                hipEventSynchronize(e1) == hipSuccess && hipEventElapsedTime(&ms, e0, e1) == hipSuccess)
                rc = PMFMM_PEAK_OK;
        }
    }
    if (rc != PMFMM_PEAK_OK) g_peak_err = "launch or timing failed";
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(out);
    if (rc == PMFMM_PEAK_OK) {
        const double fmas = (double)grid * kLanes * kChains * kUnroll * (double)iters;
        *tflops = 2.0 * fmas / (ms * 1e-3) / 1e12;
        if (ms_out) *ms_out = ms;
    }
    return rc;
}

}  // namespace

extern "C" {

int pmfmm_peak_fma(int32_t precision, int32_t iters, double* tflops, double* ms) {
    if (!tflops || iters < 16 || iters > (1 << 24) || (precision != 0 && precision != 1)) {
        g_peak_err = "need tflops != NULL, 16 <= iters <= 2^24, precision 0 or 1";
        return PMFMM_PEAK_EINVAL;
    }
    return precision == 0 ? run<double>(iters, tflops, ms) : run<float>(iters, tflops, ms);
}

const char* pmfmm_peak_last_error(void) { return g_peak_err.c_str(); }

}  // extern "C"
