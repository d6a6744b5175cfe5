// Fused inference of the learned demapper (gfx950): all weights (152 KiB of MFMA operand
// fragments + FP32 biases) live in LDS; each wavefront runs 32 received symbols through the
// three layers on v_mfma_f32_32x32x16 and writes LLRs and per-symbol GMI terms.  Layer 1 takes
// BF16 operands (features and W1 as trained); the GELU of its outputs and of layer 2's is
// evaluated two values at a time in packed FP16 (gelu2 below) and feeds layers 2 and 3 as FP16
// operands, W2 and W3 being converted from their BF16 values (exactly, above 2^-14).
//
// The hidden layers run on a quarter scale: W1, b1 and b2 are stored divided by 4 and W3
// multiplied by 4 (exact power-of-two scalings), so each hidden MFMA yields u = h / 4, the GELU
// step returns u Phi(4u) = GELU(h) / 4, and the next layer's operands absorb the factors: layer
// 2 computes W2 (a1 / 4) + b2 / 4 = h2 / 4 and layer 3 (4 W3)(a2 / 4) + b3.  The GELU then needs
// no scaling multiply of its own.
//
// Hidden units are permuted so that no activation has to move between lanes: the A operand
// of output block b (32 units) has in row i the unit
//     u(b, i) = 32 b + 16 (r / 8) + 8 h + (r % 8),  r = 4 (i / 8) + (i % 4),  h = (i / 4) % 2,
// so the MFMA result register r of a lane in half h holds unit 32 b + 16 (r / 8) + 8 h + (r % 8)
// of its symbol (column l % 32) — exactly the 8 K-slots that lane supplies as the B operand of
// the next layer's K-steps 2b (r < 8) and 2b + 1 (r >= 8).  Layer 2's output block b is
// consumed at once by layer 3's K-steps 2b and 2b + 1, so only layer 1's 16 operand fragments
// stay live.  Layer 1's bias rides in feature slots 14 and 15 (constant 1) as a BF16 hi/lo
// pair, ~16 significant bits; b2 and b3 sit in LDS in the permuted order, FP32.
#include <hip/hip_runtime.h>

#include "../../include/demap_probe.h"
#include "device_common.hpp"
#include "mlp_kernels.hpp"

namespace dm {

namespace {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(8 * sizeof(_Float16)))) _Float16 f16x8;
typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));
typedef _Float16 f16x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;

constexpr int kH = 256;
constexpr int kThreads = 512;   // 8 waves; one block per CU (the weights fill the LDS)
constexpr int kRing = 4;        // layer-2 weight fragments in flight per wave
constexpr int kW1Frags = 8 * 64;        // [block][lane]
constexpr int kW2Frags = 8 * 16 * 64;   // [block][kstep][lane]
constexpr int kW3Frags = 16 * 64;       // [kstep][lane]
constexpr int kFrags = kW1Frags + kW2Frags + kW3Frags;
constexpr int kBiasFloats = 8 * 2 * 16 + 2 * 16;  // b2 in [block][h][r] order, b3 in [h][r] order
constexpr int kLdsBytes = kFrags * 16 + kBiasFloats * 4;

__device__ __forceinline__ int perm_unit(int b, int i) {
    const int r = 4 * (i >> 3) + (i & 3);
    const int h = (i >> 2) & 1;
    return 32 * b + 16 * (r >> 3) + 8 * h + (r & 7);
}

// The tanh-form GELU on the quarter scale, u Phi(4u) for u = x / 4, Phi(x) = (1 + tanh(sqrt(2/pi)
// (x + 0.044715 x^3))) / 2, in packed FP16 with no transcendental:
//     Phi(4u) ~ clamp(1/2 + u P(u^2), 0, 1),  P(s) = p0 + p1 s + p2 s^2 + p3 s^3 + p4 s^4,
// P a near-minimax fit of (Phi(4u) - 1/2) / u on |x| <= 3.2 (the interval chosen for the
// smallest error after FP16 rounding).  Past it the odd polynomial u P(u^2) keeps growing
// (p4 > 0) and the clamp takes the factor to exactly 0 or 1, where Phi is within 1.35e-3 of it;
// very large |u| overflow u^2 to +inf, P to +inf and 1/2 + u P to +-inf, which the clamp also
// maps to 0 or 1 (no inf - inf arises).  Each step is one packed FP16 instruction for two
// values (the multiply-adds rounded once, the clamp folded into the last one): with the input
// conversion (rounding toward zero, which saturates at +-65504 instead of overflowing) and the
// final product, 8 instructions per pair; the exact form's exp2 and reciprocal alone take four
// issue cycles each per value.  Over every finite FP16 input the factor stays within 1.2e-3 of
// Phi (dm_probe_gelu checks that on the GPU against the FP64 tanh form; the fit alone is within
// 4.5e-4), and the product u Phi~ is rounded to FP16 once more.
template <class V>
__device__ __forceinline__ V gelu_quarter(V u) {
    const V zero = (V)(_Float16)0.0f, one = (V)(_Float16)1.0f;
    const V s = u * u;
    V p = (V)(_Float16)4.2214898859682375f;
    p = __builtin_elementwise_fma(p, s, (V)(_Float16)-8.968631397847826f);
    p = __builtin_elementwise_fma(p, s, (V)(_Float16)7.967970552331977f);
    p = __builtin_elementwise_fma(p, s, (V)(_Float16)-4.039456706367537f);
    p = __builtin_elementwise_fma(p, s, (V)(_Float16)1.5892242612118852f);
    const V ph = __builtin_elementwise_min(__builtin_elementwise_max(__builtin_elementwise_fma(u, p, (V)(_Float16)0.5f), zero), one);
    return u * ph;
}

// a, b: quarter-scale pre-activations h / 4; returns GELU(h) / 4 of both.
__device__ __forceinline__ f16x2 gelu2(float a, float b) {
    return gelu_quarter(__builtin_bit_cast(f16x2, __builtin_amdgcn_cvt_pkrtz(a, b)));
}

// Two pairs as one four-wide vector: each step becomes two independent packed instructions
// back to back, which keeps the VALU pipeline full without the scheduler's help.
__device__ __forceinline__ void gelu4(const float* v, f16x2& g0, f16x2& g1) {
    const f16x2 x0 = __builtin_bit_cast(f16x2, __builtin_amdgcn_cvt_pkrtz(v[0], v[1]));
    const f16x2 x1 = __builtin_bit_cast(f16x2, __builtin_amdgcn_cvt_pkrtz(v[2], v[3]));
    const f16x4 r = gelu_quarter(f16x4{x0[0], x0[1], x1[0], x1[1]});
    g0 = f16x2{r[0], r[1]};
    g1 = f16x2{r[2], r[3]};
}

// Fragment table from row-major (out x in) BF16 weights: W1t [256 x 32] (inputs 0..13 used),
// W2t [256 x 256], W3t [32 x 256]; the FP32 layer-1 bias b1 becomes input columns 14 (hi) and
// 15 (lo).  W1 and b1 are stored divided by 4 (W1 stays BF16), W3 multiplied by 4; W2 and 4 W3
// become FP16 operands, exactly for magnitudes in [2^-14, 65504], to within 2^-25 below that,
// saturated at 65504 above it.  One thread per fragment.
__device__ __forceinline__ _Float16 to_f16_sat(float w) {
    return (_Float16)fminf(fmaxf(w, -65504.0f), 65504.0f);
}

__global__ void pack_kernel(const __bf16* W1t, const __bf16* W2t, const __bf16* W3t, const float* b1, uint4* frag) {
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= kFrags) return;
    __bf16 v[8];
    _Float16 w[8];
    if (f < kW1Frags) {
        const int b = f / 64, l = f % 64;
        const int u = perm_unit(b, l % 32);
        const float bq = 0.25f * b1[u];
        const __bf16 hi = (__bf16)bq;
        const __bf16 lo = (__bf16)(bq - (float)hi);
        for (int q = 0; q < 8; ++q) {
            const int k = 8 * (l / 32) + q;
            v[q] = k == 14 ? hi : (k == 15 ? lo : (__bf16)(0.25f * (float)W1t[u * 32 + k]));
        }
    } else if (f < kW1Frags + kW2Frags) {
        const int g = f - kW1Frags;
        const int b = g / (16 * 64), t = (g / 64) % 16, l = g % 64;
        const int u = perm_unit(b, l % 32);
        for (int q = 0; q < 8; ++q) w[q] = to_f16_sat((float)W2t[u * kH + 16 * t + 8 * (l / 32) + q]);
        frag[f] = *reinterpret_cast<const uint4*>(w);
        return;
    } else {
        const int g = f - kW1Frags - kW2Frags;
        const int t = g / 64, l = g % 64;
        const int o = l % 32;
        for (int q = 0; q < 8; ++q) w[q] = to_f16_sat(4.0f * (float)W3t[o * kH + 16 * t + 8 * (l / 32) + q]);
        frag[f] = *reinterpret_cast<const uint4*>(w);
        return;
    }
    frag[f] = *reinterpret_cast<const uint4*>(v);
}

__global__ __launch_bounds__(kThreads) void mlp_infer_kernel(const MlpInferArgs a) {
    extern __shared__ uint4 lds[];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6, h = lane >> 5, j = lane & 31;
    float* lbias = reinterpret_cast<float*>(lds + kFrags);
    for (int i = tid; i < kFrags; i += kThreads) lds[i] = a.frag[i];
    // b2 as [block][h][r]: unit 32b + 16(r/8) + 8h + (r%8); b3 as [h][r]: output 8(r/4) + 4h + (r%4)
    for (int i = tid; i < 8 * 2 * 16; i += kThreads) {
        const int b = i / 32, hh = (i / 16) % 2, r = i % 16;
        lbias[i] = 0.25f * a.bias[kH + 32 * b + 16 * (r >> 3) + 8 * hh + (r & 7)];  // b2 / 4
    }
    for (int i = tid; i < 32; i += kThreads) {
        const int hh = i / 16, r = i % 16;
        lbias[8 * 2 * 16 + i] = a.bias[2 * kH + 8 * (r >> 2) + 4 * hh + (r & 3)];
    }
    __syncthreads();
    const uint4* w1 = lds;
    const uint4* w2 = lds + kW1Frags;
    const uint4* w3 = lds + kW1Frags + kW2Frags;

    if (a.N <= 0) return;  // the clamped loads below need a row 0 (callers skip empty ranges)
    const int64_t tiles = (a.N + 31) / 32;
    const int slot = (blockIdx.x * (kThreads / 64) + wave) % kAccSlots;
    double gsum = 0.0;
    const int64_t stride = (int64_t)gridDim.x * (kThreads / 64);
    // A tile's received values and transmitted rows are loaded one tile ahead, so their memory
    // latency overlaps the previous tile's layers.
    // The loads are unconditional (indices clamped into the arrays, N >= 1 here) and their
    // values are masked only where they are used, a tile later: a load under a branch, or
    // selected right away, would make the compiler wait for it at once.
    float yv[8];
    uint32_t txr = 0;
    bool yact = false;
    auto fetch = [&](int64_t tt) {
        const int64_t nn = tt * 32 + j;
        yact = nn < a.N;  // false past the last tile too
        const size_t nc = (size_t)(yact ? nn : a.N - 1);
#pragma unroll
        for (int q = 0; q < 8; ++q) yv[q] = a.y[nc * a.D + min(8 * h + q, a.D - 1)];
        if (a.tx) txr = a.tx[nc];
    };
    fetch((int64_t)blockIdx.x * (kThreads / 64) + wave);
    for (int64_t t = (int64_t)blockIdx.x * (kThreads / 64) + wave; t < tiles; t += stride) {
        const int64_t n = t * 32 + j;
        const bool active = n < a.N;
        // features: slot k = 8h + q; k < D: y, k == D: SNR feature, k = 14, 15: 1 (bias), else 0
        bf16x8 xf;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int k = 8 * h + q;
            float v = 0.0f;
            if (k < a.D) v = yact ? yv[q] : 0.0f;
            else if (k == a.D) v = a.snr_feature;
            else if (k >= 14) v = 1.0f;
            xf[q] = (__bf16)v;
        }
        uint32_t row_cur = yact ? txr : 0u;
        {
            // the values above are consumed before the next loads issue (the empty asm keeps
            // the selects from sinking below them): a wait the compiler places for the values
            // must not also cover those loads
            uint4 xb = __builtin_bit_cast(uint4, xf);
            asm volatile("" : "+v"(xb.x), "+v"(xb.y), "+v"(xb.z), "+v"(xb.w), "+v"(row_cur)::"memory");
            xf = __builtin_bit_cast(bf16x8, xb);
        }
        // label of the transmitted point, read now and used after layer 3
        int txl = 0;
        if (a.tx) {
            uint32_t row = row_cur;
            if (row >= (uint32_t)a.M) {
                if (a.bad_tx) atomicOr(a.bad_tx, 1u);
                row = 0;
            }
            txl = a.row2label[row];
        }
        fetch(t + stride);
        // Two GELU pairs (two independent chains the scheduler interleaves) pinned where they
        // are written: without the empty asm the compiler sinks them to their first use and the
        // VALU work bunches up behind the MFMAs.
        auto gelu4_here = [&](const float* v, f16x2& g0, f16x2& g1) {
            gelu4(v, g0, g1);
            uint32_t b0 = __builtin_bit_cast(uint32_t, g0);
            uint32_t b1 = __builtin_bit_cast(uint32_t, g1);
            asm volatile("" : "+v"(b0), "+v"(b1));
            g0 = __builtin_bit_cast(f16x2, b0);
            g1 = __builtin_bit_cast(f16x2, b1);
        };
        f16x8 a1[16];
        f32x16 acc3 = {};
        // Layer-2 weight fragments stream through a ring of kRing registers: the read of
        // fragment g + kRing is issued right after fragment g is consumed, so LDS latency
        // overlaps kRing - 1 MFMAs (the ring runs on across blocks; past the end it rereads the
        // last fragment, which is never used).  The layer is software-pipelined over its 8 output
        // blocks: while the 16 MFMAs of block b run, the wave evaluates block b-1's 16 GELUs, one
        // pair per two MFMAs, and feeds them to layer 3 afterwards, so matrix and vector work
        // overlap within the wave.  Layer 1 is folded into layer 2's first block the same way:
        // layer-1 block b + 1's MFMA is issued before block b's GELUs, and layer-2 k-steps 2b and
        // 2b + 1 run as soon as those GELUs have produced their operands.
        f16x8 ring[kRing];
#pragma unroll
        for (int q = 0; q < kRing; ++q) ring[q] = __builtin_bit_cast(f16x8, w2[q * 64 + lane]);
        auto l2_step = [&](int b, int ks, f32x16 acc) {
            const f16x8 cur = ring[ks % kRing];
            const int next = min(b * 16 + ks + kRing, 8 * 16 - 1);
            ring[ks % kRing] = __builtin_bit_cast(f16x8, w2[next * 64 + lane]);
            return __builtin_amdgcn_mfma_f32_32x32x16_f16(cur, a1[ks], acc, 0, 0, 0);
        };
        // Block p's layer-2 biases seed its accumulators (the MFMAs add onto them).
        auto bias_acc = [&](int p) {
            const float4* bb4 = reinterpret_cast<const float4*>(lbias + (p * 2 + h) * 16);
            f32x16 acc;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const float4 v = bb4[q];
                acc[4 * q] = v.x;
                acc[4 * q + 1] = v.y;
                acc[4 * q + 2] = v.z;
                acc[4 * q + 3] = v.w;
            }
            return acc;
        };
        auto l1_mfma = [&](int b) {
            return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, w1[b * 64 + lane]), xf,
                                                           f32x16{}, 0, 0, 0);
        };
        f32x16 accp = bias_acc(0);
        f32x16 acc1 = l1_mfma(0);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            f32x16 acc1n = {};
            if (b < 7) acc1n = l1_mfma(b + 1);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int half = 0; half < 2; ++half) {
#pragma unroll
                for (int r = 8 * half; r < 8 * half + 8; r += 4) {
                    const float v[4] = {acc1[r], acc1[r + 1], acc1[r + 2], acc1[r + 3]};
                    f16x2 g0, g1;
                    gelu4_here(v, g0, g1);
                    a1[2 * b + half][r & 7] = g0[0];
                    a1[2 * b + half][(r & 7) + 1] = g0[1];
                    a1[2 * b + half][(r & 7) + 2] = g1[0];
                    a1[2 * b + half][(r & 7) + 3] = g1[1];
                }
                accp = l2_step(0, 2 * b + half, accp);
                __builtin_amdgcn_sched_barrier(0);  // keep the read kRing steps ahead of its use
            }
            acc1 = acc1n;
        }
        // block p's GELUs feed layer 3; with `next` the MFMAs of block p + 1 run in between
        auto finish = [&](int p, bool next, f32x16& accn) {
            const f16x8 w3lo = __builtin_bit_cast(f16x8, w3[(2 * p) * 64 + lane]);
            const f16x8 w3hi = __builtin_bit_cast(f16x8, w3[(2 * p + 1) * 64 + lane]);
            f16x8 lo, hi;
#pragma unroll
            for (int ks = 0; ks < 16; ++ks) {
                if (next) accn = l2_step(p + 1, ks, accn);
                if ((ks & 3) == 3) {
                    const float v[4] = {accp[ks - 3], accp[ks - 2], accp[ks - 1], accp[ks]};
                    f16x2 g0, g1;
                    if (next) {
                        gelu4_here(v, g0, g1);
                    } else {
                        gelu4(v, g0, g1);
                    }
                    f16x8& dst = ks < 8 ? lo : hi;
                    dst[(ks & 7) - 3] = g0[0];
                    dst[(ks & 7) - 2] = g0[1];
                    dst[(ks & 7) - 1] = g1[0];
                    dst[ks & 7] = g1[1];
                }
                // one MFMA and its ring read per step, two GELU pairs every fourth step: the read
                // stays kRing steps ahead of its use and the GELUs spread over the MFMAs
                if (next) __builtin_amdgcn_sched_barrier(0);
            }
            acc3 = __builtin_amdgcn_mfma_f32_32x32x16_f16(w3lo, lo, acc3, 0, 0, 0);
            acc3 = __builtin_amdgcn_mfma_f32_32x32x16_f16(w3hi, hi, acc3, 0, 0, 0);
        };
        // Waves w and w + 4 share a SIMD.  During the MFMA-bound blocks a raised wave priority
        // lets this wave's matrix instructions issue ahead of the other wave's vector work, which
        // then fills the gaps (measured: +2% over equal priorities).
        __builtin_amdgcn_s_setprio(1);
#pragma unroll
        for (int b = 1; b < 8; ++b) {
            f32x16 accn = bias_acc(b);
            finish(b - 1, true, accn);
            accp = accn;
        }
        __builtin_amdgcn_s_setprio(0);
        {
            f32x16 unused = {};
            finish(7, false, unused);
        }
        // outputs: register r holds output o = 8 (r / 4) + 4 h + (r % 4) of symbol n
        const float* b3 = lbias + 8 * 2 * 16 + h * 16;
        float g = 0.0f;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int o = 8 * (r >> 2) + 4 * h + (r & 3);
            if (o < a.m) {
                const float lam = acc3[r] + b3[r];
                if (a.llr && active) a.llr[(size_t)n * a.m + o] = lam;
                g += gmi_bit_term(lam * 1.4426950408889634f, (txl >> (a.m - 1 - o)) & 1);
            }
        }
        gsum += active ? (double)g : 0.0;
    }
    if (a.acc) {
        gsum = wave_sum(gsum);
        if (lane == 0) acc_add(a.acc, 0, slot, 0, gsum);
    }
}

__global__ void probe_gelu_kernel(const float* x, float* out, int64_t n) {
    const int64_t i = 2 * ((int64_t)blockIdx.x * blockDim.x + threadIdx.x);
    if (i >= n) return;
    const f16x2 g = gelu2(0.25f * x[i], i + 1 < n ? 0.25f * x[i + 1] : 0.0f);
    out[i] = 4.0f * (float)g[0];
    if (i + 1 < n) out[i + 1] = 4.0f * (float)g[1];
}

}  // namespace

size_t mlp_frag_count() { return kFrags; }

hipError_t launch_mlp_pack(const __bf16* W1t, const __bf16* W2t, const __bf16* W3t, const float* b1, uint4* frag,
                           hipStream_t st) {
    hipLaunchKernelGGL(pack_kernel, dim3((kFrags + 255) / 256), dim3(256), 0, st, W1t, W2t, W3t, b1, frag);
    return hipGetLastError();
}

hipError_t prepare_mlp_infer() {
    return hipFuncSetAttribute((const void*)mlp_infer_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBytes);
}

hipError_t launch_mlp_infer(const MlpInferArgs& a, int grid, hipStream_t st) {
    hipLaunchKernelGGL(mlp_infer_kernel, dim3(grid), dim3(kThreads), kLdsBytes, st, a);
    return hipGetLastError();
}

}  // namespace dm

extern "C" int dm_probe_gelu(const float* x, float* out, int64_t n) {
    if (n < 0 || n > (int64_t(1) << 24) || (n > 0 && (!x || !out))) return -1;
    if (n == 0) return 0;
    float *dx = nullptr, *dy = nullptr;
    if (hipMalloc(&dx, n * 4) != hipSuccess || hipMalloc(&dy, n * 4) != hipSuccess) {
        hipFree(dx);
        return -4;
    }
    hipError_t e = hipMemcpy(dx, x, n * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) {
        const int64_t pairs = (n + 1) / 2;
        hipLaunchKernelGGL(dm::probe_gelu_kernel, dim3((unsigned)((pairs + 255) / 256)), dim3(256), 0, 0, dx, dy, n);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpy(out, dy, n * 4, hipMemcpyDeviceToHost);
    hipFree(dx);
    hipFree(dy);
    return e == hipSuccess ? 0 : -3;
}
