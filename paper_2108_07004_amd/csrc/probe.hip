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

// ---- device-scope atomics on one address and spread over the fix-up queue's counters ----
namespace {

constexpr int kAtomThreads = 1024;
constexpr int kAtomPerWave = 32;
constexpr int kAtomAddrs = 64;    // as many addresses as the fix-up queue has counters
constexpr int kAtomStride = 64;   // words between two of them, as in the queue

// Lane 0 of every wave adds kAtomPerWave times to counter (global wave index) % naddr.
__global__ __launch_bounds__(kAtomThreads) void probe_atomics(unsigned int* ctr, int naddr) {
    const unsigned int w = blockIdx.x * (kAtomThreads / 64) + (threadIdx.x >> 6);
    unsigned int* c = ctr + (size_t)(w % (unsigned int)naddr) * kAtomStride;
    if ((threadIdx.x & 63) == 0)
        for (int i = 0; i < kAtomPerWave; ++i) atomicAdd(c, 1u);
}

double time_atomics(unsigned int* ctr, int naddr, int grid, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
    hipLaunchKernelGGL(probe_atomics, dim3(grid), dim3(kAtomThreads), 0, st, ctr, naddr);  // warm-up
    hipEventRecord(e0, st);
    hipLaunchKernelGGL(probe_atomics, dim3(grid), dim3(kAtomThreads), 0, st, ctr, naddr);
    hipEventRecord(e1, st);
    hipEventSynchronize(e1);
    float ms = 0.0f;
    hipEventElapsedTime(&ms, e0, e1);
    return (double)ms * 1e-3;
}

}  // namespace

extern "C" int dm_probe_atomic_rates(double* rates, void* stream) {
    if (!rates) return -1;
    hipStream_t st = (hipStream_t)stream;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return -3;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return -3;
    unsigned int* ctr = nullptr;
    if (hipMalloc(&ctr, sizeof(unsigned int) * kAtomAddrs * kAtomStride) != hipSuccess) return -4;
    hipEvent_t e0, e1;
    hipEventCreate(&e0);
    hipEventCreate(&e1);
    const double n = (double)cus * (kAtomThreads / 64) * kAtomPerWave;
    const double t_one = time_atomics(ctr, 1, cus, st, e0, e1);
    const double t_spread = time_atomics(ctr, kAtomAddrs, cus, st, e0, e1);
    hipError_t err = hipGetLastError();
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    hipFree(ctr);
    if (err != hipSuccess) return -3;
    rates[0] = n / t_one;     // atomics per second, all on one address
    rates[1] = n / t_spread;  // atomics per second over kAtomAddrs addresses
    rates[2] = (double)kAtomAddrs;
    return 0;
}

// ---- MFMA lane-layout check (gfx950): one 32x32x16 or 16x16x32 product with the fragment
// mapping the demapping kernels assume, so a test can compare it with A @ B on the host.
namespace {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8_t;
typedef __attribute__((__vector_size__(8 * sizeof(_Float16)))) _Float16 f16x8_t;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16_t;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4_t;

template <typename T, typename V>
__global__ __launch_bounds__(64) void probe_mfma_layout(const float* A, const float* B, float* Dm, int shape) {
    const int l = threadIdx.x;
    V a, b;
    if (shape == 0) {  // 32x32x16: A 32x16 row-major, B 16x32 row-major, D 32x32
        for (int v = 0; v < 8; ++v) {
            a[v] = (T)A[(l % 32) * 16 + 8 * (l / 32) + v];
            b[v] = (T)B[(8 * (l / 32) + v) * 32 + (l % 32)];
        }
        f32x16_t d = {};
        if constexpr (sizeof(T) == 2 && __is_same(T, __bf16)) d = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, d, 0, 0, 0);
        else d = __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, d, 0, 0, 0);
        for (int r = 0; r < 16; ++r) Dm[(8 * (r / 4) + 4 * (l / 32) + (r % 4)) * 32 + (l % 32)] = d[r];
    } else {  // 16x16x32: A 16x32, B 32x16, D 16x16
        for (int v = 0; v < 8; ++v) {
            a[v] = (T)A[(l % 16) * 32 + 8 * (l / 16) + v];
            b[v] = (T)B[(8 * (l / 16) + v) * 16 + (l % 16)];
        }
        f32x4_t d = {};
        if constexpr (__is_same(T, __bf16)) d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, d, 0, 0, 0);
        else d = __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, d, 0, 0, 0);
        for (int r = 0; r < 4; ++r) Dm[(4 * (l / 16) + r) * 16 + (l % 16)] = d[r];
    }
}

}  // namespace

extern "C" int dm_probe_mfma_layout(int dtype, int shape, const float* A, const float* B, float* Dout) {
    if (!A || !B || !Dout || (dtype != 0 && dtype != 1) || (shape != 0 && shape != 1)) return -1;
    const size_t na = 512, nb = 512, nd = shape == 0 ? 1024 : 256;
    float *dA = nullptr, *dB = nullptr, *dD = nullptr;
    if (hipMalloc(&dA, na * 4) != hipSuccess || hipMalloc(&dB, nb * 4) != hipSuccess ||
        hipMalloc(&dD, nd * 4) != hipSuccess) {
        hipFree(dA);
        hipFree(dB);
        return -4;
    }
    hipMemcpy(dA, A, na * 4, hipMemcpyHostToDevice);
    hipMemcpy(dB, B, nb * 4, hipMemcpyHostToDevice);
    if (dtype == 0) hipLaunchKernelGGL((probe_mfma_layout<__bf16, bf16x8_t>), dim3(1), dim3(64), 0, 0, dA, dB, dD, shape);
    else hipLaunchKernelGGL((probe_mfma_layout<_Float16, f16x8_t>), dim3(1), dim3(64), 0, 0, dA, dB, dD, shape);
    hipError_t e = hipMemcpy(Dout, dD, nd * 4, hipMemcpyDeviceToHost);
    hipFree(dA);
    hipFree(dB);
    hipFree(dD);
    return e == hipSuccess ? 0 : -3;
}
