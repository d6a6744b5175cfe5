// Throughput probes of the vector ALU on the current GPU: the rates that bound the exact
// demapper (one exp2 per symbol-point pair plus the subset-sum adds).
#include <hip/hip_runtime.h>

#include "../../include/demap_probe.h"

namespace {

constexpr int kChains = 16;   // independent dependency chains per lane
constexpr int kIters = 4096;  // iterations per lane
constexpr int kThreads = 256;

// Pure exp2: x <- 2^(-x) on every chain (converges near 0.64, no overflow).
__global__ __launch_bounds__(kThreads) void probe_exp2(float* out, float seed) {
    float x[kChains];
#pragma unroll
    for (int i = 0; i < kChains; ++i) x[i] = seed + 1e-3f * (threadIdx.x + i);
    for (int it = 0; it < kIters; ++it) {
#pragma unroll
        for (int i = 0; i < kChains; ++i) x[i] = __builtin_amdgcn_exp2f(-x[i]);
    }
    float s = 0.0f;
#pragma unroll
    for (int i = 0; i < kChains; ++i) s += x[i];
    if (s == 12345.0f) out[threadIdx.x] = s;  // keeps the work alive
}

// Full-rate FMA: x <- x * a + b.
__global__ __launch_bounds__(kThreads) void probe_fma(float* out, float seed) {
    float x[kChains];
#pragma unroll
    for (int i = 0; i < kChains; ++i) x[i] = seed + 1e-3f * (threadIdx.x + i);
    const float a = 0.999f + seed * 1e-9f, b = 1e-4f;
    for (int it = 0; it < kIters; ++it) {
#pragma unroll
        for (int i = 0; i < kChains; ++i) x[i] = fmaf(x[i], a, b);
    }
    float s = 0.0f;
#pragma unroll
    for (int i = 0; i < kChains; ++i) s += x[i];
    if (s == 12345.0f) out[threadIdx.x] = s;
}

// The exact demapper's inner step: e = 2^t, acc += e, T += e (one exp2, two adds).
__global__ __launch_bounds__(kThreads) void probe_exp2_add2(float* out, float seed) {
    float t[kChains], acc[kChains], T = 0.0f;
#pragma unroll
    for (int i = 0; i < kChains; ++i) {
        t[i] = -(seed + 1e-3f * (threadIdx.x + i));
        acc[i] = 0.0f;
    }
    for (int it = 0; it < kIters; ++it) {
#pragma unroll
        for (int i = 0; i < kChains; ++i) {
            const float e = __builtin_amdgcn_exp2f(t[i]);
            acc[i] += e;
            T += e;
            t[i] = -e;  // source-negation modifier: no extra instruction
        }
    }
    float s = T;
#pragma unroll
    for (int i = 0; i < kChains; ++i) s += acc[i];
    if (s == 12345.0f) out[threadIdx.x] = s;
}

template <typename K>
double time_kernel(K kern, float* out, int grid, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
    hipLaunchKernelGGL(kern, dim3(grid), dim3(kThreads), 0, st, out, 0.5f);  // warm-up
    hipEventRecord(e0, st);
    hipLaunchKernelGGL(kern, dim3(grid), dim3(kThreads), 0, st, out, 0.25f);
    hipEventRecord(e1, st);
    hipEventSynchronize(e1);
    float ms = 0.0f;
    hipEventElapsedTime(&ms, e0, e1);
    return (double)ms * 1e-3;
}

}  // namespace

extern "C" int dm_probe_valu_rates(double* rates, void* stream) {
    if (!rates) return -1;
    hipStream_t st = (hipStream_t)stream;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return -3;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return -3;
    float* out = nullptr;
    if (hipMalloc(&out, kThreads * sizeof(float)) != hipSuccess) return -4;
    hipEvent_t e0, e1;
    hipEventCreate(&e0);
    hipEventCreate(&e1);
    const int grid = cus * 32;  // 32 blocks of 4 waves per CU: enough waves to hide latency
    const double lanes = (double)grid * kThreads * kChains * kIters;
    const double t_exp = time_kernel(probe_exp2, out, grid, st, e0, e1);
    const double t_fma = time_kernel(probe_fma, out, grid, st, e0, e1);
    const double t_mix = time_kernel(probe_exp2_add2, out, grid, st, e0, e1);
    hipError_t err = hipGetLastError();
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    hipFree(out);
    if (err != hipSuccess) return -3;
    rates[0] = lanes / t_exp;   // exp2 lane-ops per second
    rates[1] = lanes / t_fma;   // fma lane-ops per second
    rates[2] = lanes / t_mix;   // (exp2 + 2 add) steps per second
    rates[3] = (double)cus;
    return 0;
}
