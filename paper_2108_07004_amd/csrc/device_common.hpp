// Device-side helpers and launch-argument layout shared by the demapping kernels (gfx950).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dm {

constexpr int kMaxSnrPerLaunch = 32;  // SNR points per launch (kernel-argument block stays < 1 KiB)
constexpr int kAccSlots = 64;         // fixed-point accumulator slots per SNR point (spreads atomics)
constexpr double kFixScale = 268435456.0;  // 2^28: GMI/MI sums are accumulated as int64 * 2^-28
constexpr uint32_t kMiFlag = 0x80000000u;  // fix-up mask bit: recompute the MI term

// One symbol whose far-subset sums underflowed the shared exponent window.
struct FixEntry {
    uint32_t n;     // symbol index within the block
    uint32_t snr;   // SNR index within the launch
    uint32_t mask;  // bit p set: recompute label bit p; kMiFlag: recompute the MI term
    uint32_t pad;
};

struct SnrArg {
    const float* y;  // N x D received block
    float* llr;      // N x m output or null
    float c;         // log2(e) / (2 sigma2), rounded once from FP64
    int32_t pad;
};

struct LaunchArgs {
    const float* table;          // M x D FP32 points in label order (row j has label j)
    const uint16_t* row2label;   // M: label of each caller row
    const uint16_t* tx;          // N transmitted caller rows, or null (no GMI/MI)
    int64_t N;
    int64_t tiles_per_snr;
    int32_t M, D, m, n_snr;
    float K;                     // exponent offset: e_j = 2^(K - c ||y - x_j||^2)
    float flag_thresh;           // 2^(m-102): a subset sum below this is recomputed
    float near_thresh;           // 2^(m-42): GMI-only shortcut bound for the near subset
    int32_t want_llr;
    unsigned long long* acc;     // [n_snr][kAccSlots][2] int64 fixed-point GMI / MI sums
    uint32_t* fix_pairs;         // [n_snr] count of (symbol, bit) pairs sent to the fix-up
    uint32_t* bad_tx;            // set to 1 when a transmitted index is >= M (clamped, reported)
    FixEntry* queue;
    uint32_t* queue_count;
    uint32_t queue_cap;
    SnrArg snr[kMaxSnrPerLaunch];
};

// Label of the transmitted row; an out-of-range row is clamped and reported.
__device__ __forceinline__ int tx_label(const LaunchArgs& a, int64_t n) {
    uint32_t r = a.tx[n];
    if (r >= (uint32_t)a.M) {
        if (a.bad_tx) atomicOr(a.bad_tx, 1u);
        r = 0;
    }
    return (int)a.row2label[r];
}

__device__ __forceinline__ float hw_exp2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ float hw_log2(float x) { return __builtin_amdgcn_logf(x); }

// log2(a) - log2(b) with exact binary exponents: the mantissa logs are O(1), so the
// result keeps FP32 accuracy even when both logs are ~100 (the exponent offset K).
__device__ __forceinline__ float log2_ratio(float a, float b) {
    const int ea = __builtin_amdgcn_frexp_expf(a);
    const int eb = __builtin_amdgcn_frexp_expf(b);
    const float ma = __builtin_amdgcn_frexp_mantf(a);
    const float mb = __builtin_amdgcn_frexp_mantf(b);
    return (float)(ea - eb) + (hw_log2(ma) - hw_log2(mb));
}

// log2(1 + u) for u in [0, 1]; the series branch keeps the tiny-u tail that 1+u would lose.
__device__ __forceinline__ float log2_1p(float u) {
    return (u < 0x1p-12f) ? u * (1.44269504088896341f - 0.72134752044448170f * u) : hw_log2(1.0f + u);
}

// Per-bit GMI term 1 - log2(1 + 2^(s L)), L the LLR in log2 units, s = +1 for a
// transmitted 0 and -1 for a transmitted 1.
__device__ __forceinline__ float gmi_bit_term(float L, int tx_bit) {
    const float x = tx_bit ? -L : L;
    return 1.0f - (fmaxf(x, 0.0f) + log2_1p(hw_exp2(-fabsf(x))));
}

// Butterfly sum over the 64 lanes of a wavefront, FP64, fixed order (every lane gets the sum).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ void acc_add(unsigned long long* acc, int snr, int slot, int which, double v) {
    const long long q = __double2ll_rn(v * kFixScale);
    if (q != 0) atomicAdd(acc + ((size_t)snr * kAccSlots + slot) * 2 + which, (unsigned long long)q);
}

// Direct squared distance ||y - x||^2 in FP32 (differences first, then squares).
template <int D>
__device__ __forceinline__ float sqdist(const float (&y)[D], const float* x) {
    float acc = 0.0f;
#pragma unroll
    for (int d = 0; d < D; ++d) {
        const float t = y[d] - x[d];
        acc = fmaf(t, t, acc);
    }
    return acc;
}

}  // namespace dm
