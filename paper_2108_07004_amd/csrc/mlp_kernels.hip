// Kernels of the learned demapper: an MLP (D+1) -> H -> H -> m with GELU, BF16 weights and
// activations, FP32 accumulation on v_mfma_f32_32x32x16_bf16 (gfx950).
//
// Training runs one NT GEMM kernel, C[M x N] = A[M x K] . Bt[N x K]^T with both operands
// K-contiguous (row-major A, row-major Bt), one wavefront per 32 x 32 output tile and an
// optional split of K, followed by a fused epilogue:
//   PARTIAL      FP32 partial sums part[split][M][N] (weight gradients over the batch);
//   FWD_HIDDEN   h = acc + b; H = h (FP32); a = gelu(h) stored row-major and transposed;
//   FWD_OUT      o = acc + b; dO = (sigmoid(o) - sigmoid(t)) / (B m) stored row-major and
//                transposed, and the soft-BCE loss summed per tile;
//   BWD_HIDDEN   dh = acc * gelu'(H) stored row-major and transposed.
// Gradients are then reduced over the K splits in a fixed order (deterministic) and Adam
// updates the FP32 master weights and rewrites their BF16 copies.
//
// Activations and back-propagated deltas are stored as BF16 pairs hi + lo (lo = the rounding
// remainder, about 16 significant bits together) and enter every product that reads them as
// such: hi.b + lo.b, or hi.hi + hi.lo + lo.hi when both operands are pairs.  Only the weights
// (BF16 copies of the FP32 masters) and the network inputs are single BF16 words, so the
// gradients are those of the network on BF16-rounded weights and inputs, with activations and
// deltas carried to about 2^-16 relative instead of BF16's 2^-8.
#include <hip/hip_runtime.h>

#include "mlp_kernels.hpp"

namespace dm {

namespace {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;

__device__ __forceinline__ float rcp_f(float x) { return __builtin_amdgcn_rcpf(x); }

__device__ __forceinline__ float gelu_f(float x) {
    // 0.5 x (1 + tanh(u)) = x * sigmoid(2u), u = sqrt(2/pi) (x + 0.044715 x^3)
    const float u2 = 1.5957691216057308f * x * fmaf(0.044715f, x * x, 1.0f);
    return x * rcp_f(1.0f + __builtin_amdgcn_exp2f(-1.4426950408889634f * u2));
}

__device__ __forceinline__ float gelu_grad_f(float x) {
    const float x2 = x * x;
    const float u2 = 1.5957691216057308f * x * fmaf(0.044715f, x2, 1.0f);  // 2u
    const float s = rcp_f(1.0f + __builtin_amdgcn_exp2f(-1.4426950408889634f * u2));  // sigmoid(2u)
    // d/dx [x sigmoid(2u)] = s + x s (1 - s) d(2u)/dx,  d(2u)/dx = 2 sqrt(2/pi) (1 + 3 * 0.044715 x^2)
    return s + x * s * (1.0f - s) * 1.5957691216057308f * fmaf(0.134145f, x2, 1.0f);
}

__device__ __forceinline__ float sigmoid_f(float x) { return rcp_f(1.0f + __builtin_amdgcn_exp2f(-1.4426950408889634f * x)); }

__device__ __forceinline__ float softplus_f(float x) {
    return fmaxf(x, 0.0f) + 0.69314718055994531f * __builtin_amdgcn_logf(1.0f + __builtin_amdgcn_exp2f(-1.4426950408889634f * fabsf(x)));
}

// Stores v as a BF16 pair: hi[idx] = bf16(v), lo[idx] = bf16(v - hi) (the difference is exact
// in FP32); lo may be null.
__device__ __forceinline__ void store_pair(__bf16* hi, __bf16* lo, size_t idx, float v) {
    const __bf16 h = (__bf16)v;
    hi[idx] = h;
    if (lo) lo[idx] = (__bf16)(v - (float)h);
}

template <bool ALO, bool BLO>
__global__ __launch_bounds__(256) void gemm_nt_kernel(const GemmArgs g) {
    const int lane = threadIdx.x & 63;
    const int wave = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int tiles_m = g.M / 32, tiles_n = g.N / 32;
    const int tiles = tiles_m * tiles_n;
    if (wave >= tiles * g.splits) return;  // whole wavefront exits together
    const int split = wave / tiles;
    const int tile = wave % tiles;
    const int m0 = (tile / tiles_n) * 32, n0 = (tile % tiles_n) * 32;
    const int kc = g.K / g.splits;
    const int k_begin = split * kc, k_end = k_begin + kc;
    const int r = lane & 31, h = lane >> 5;
    const size_t aoff = (size_t)(m0 + r) * g.lda + 8 * h;
    const size_t boff = (size_t)(n0 + r) * g.ldb + 8 * h;
    f32x16 acc = {};
    for (int k = k_begin; k < k_end; k += 16) {
        const bf16x8 a = *reinterpret_cast<const bf16x8*>(g.A + aoff + k);
        const bf16x8 b = *reinterpret_cast<const bf16x8*>(g.Bt + boff + k);
        if constexpr (ALO) {
            const bf16x8 al = *reinterpret_cast<const bf16x8*>(g.A_lo + aoff + k);
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, b, acc, 0, 0, 0);
        }
        if constexpr (BLO) {
            const bf16x8 bl = *reinterpret_cast<const bf16x8*>(g.Bt_lo + boff + k);
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, bl, acc, 0, 0, 0);
        }
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
    }
    const int j = n0 + r;  // output column of this lane
    float loss = 0.0f;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int i = m0 + 8 * (q >> 2) + 4 * h + (q & 3);  // output row of register q
        const float v = acc[q];
        switch (g.epi) {
            case kEpiPartial:
                g.part[((size_t)split * g.M + i) * g.N + j] = v;
                break;
            case kEpiFwdHidden: {
                const float hv = v + g.bias[j];
                g.Hout[(size_t)i * g.ldh + j] = hv;
                const float a = gelu_f(hv);
                store_pair(g.Aout, g.Aout_lo, (size_t)i * g.ldo + j, a);
                store_pair(g.AoutT, g.AoutT_lo, (size_t)j * g.ldt + i, a);
                break;
            }
            case kEpiFwdOut: {
                float d = 0.0f;
                if (j < g.mout) {
                    const float o = v + g.bias[j];
                    const float t = g.target[(size_t)i * g.ld_target + j];
                    const float p = sigmoid_f(t);
                    d = (sigmoid_f(o) - p) * g.scale;
                    loss += (softplus_f(o) - p * o) - (softplus_f(t) - p * t);
                    if (g.Hout) g.Hout[(size_t)i * g.ldh + j] = o;
                }
                store_pair(g.Aout, g.Aout_lo, (size_t)i * g.ldo + j, d);
                store_pair(g.AoutT, g.AoutT_lo, (size_t)j * g.ldt + i, d);
                break;
            }
            case kEpiBwdHidden: {
                const float d = v * gelu_grad_f(g.Hin[(size_t)i * g.ldh + j]);
                if (g.Aout) store_pair(g.Aout, g.Aout_lo, (size_t)i * g.ldo + j, d);
                store_pair(g.AoutT, g.AoutT_lo, (size_t)j * g.ldt + i, d);
                break;
            }
        }
    }
    if (g.epi == kEpiFwdOut && g.loss_tiles) {
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) loss += __shfl_xor(loss, off, 64);
        if (lane == 0) g.loss_tiles[tile] = loss;
    }
}

// Row sums of a BF16 matrix (rows contiguous): out[row] = sum_b X[row][b] (+ Xlo[row][b]).
__global__ __launch_bounds__(256) void rowsum_kernel(const __bf16* X, const __bf16* Xlo, int rows, int cols, int ld,
                                                     float* out) {
    // One workgroup per row; 16-byte loads of 8 values when the row layout allows; fixed
    // summation order (per thread, then the wave butterfly, then the 4 waves in order).
    const int row = blockIdx.x;
    if (row >= rows) return;
    const size_t roff = (size_t)row * ld;
    float s = 0.0f;
    const bool vec = (cols % 8 == 0) && (ld % 8 == 0) && ((reinterpret_cast<uintptr_t>(X) & 15) == 0) &&
                     ((reinterpret_cast<uintptr_t>(Xlo) & 15) == 0);
    if (vec) {
        for (int c = threadIdx.x * 8; c < cols; c += blockDim.x * 8) {
            const bf16x8 v = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(X + roff + c));
            if (Xlo) {
                const bf16x8 l = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(Xlo + roff + c));
#pragma unroll
                for (int q = 0; q < 8; ++q) s += (float)v[q] + (float)l[q];
            } else {
#pragma unroll
                for (int q = 0; q < 8; ++q) s += (float)v[q];
            }
        }
    } else {
        for (int c = threadIdx.x; c < cols; c += blockDim.x) s += (float)X[roff + c] + (Xlo ? (float)Xlo[roff + c] : 0.0f);
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
    __shared__ float part[4];
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) out[row] = (part[0] + part[1]) + (part[2] + part[3]);
}

// grad[idx] = sum over splits (fixed order) of part[s][idx] for idx < n.
__global__ void reduce_splits_kernel(const float* part, int splits, size_t n, float* grad) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        float s = 0.0f;
        int k = 0;
        for (; k + 8 <= splits; k += 8) {  // eight loads in flight, added in split order
            float v[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) v[q] = part[(size_t)(k + q) * n + i];
#pragma unroll
            for (int q = 0; q < 8; ++q) s += v[q];
        }
        for (; k < splits; ++k) s += part[(size_t)k * n + i];
        grad[i] = s;
    }
}

// Adam on one parameter tensor (rows x cols, row-major FP32 master), then BF16 copies:
// copy (rows x cols row-major) and copyT (cols x rows), either may be null.  mask_rows /
// mask_cols: entries outside [0, mask_rows) x [0, mask_cols) are padding and stay zero.
__device__ __forceinline__ void adam_element(const AdamArgs& a, size_t i) {
    const int rr = (int)(i / a.cols), cc = (int)(i % a.cols);
    float w = a.w[i];
    if (rr < a.mask_rows && cc < a.mask_cols) {
        const float g = a.grad[i];
        const float m = a.beta1 * a.m[i] + (1.0f - a.beta1) * g;
        const float v = a.beta2 * a.v[i] + (1.0f - a.beta2) * g * g;
        a.m[i] = m;
        a.v[i] = v;
        const float mh = m / a.bc1, vh = v / a.bc2;
        w -= a.lr * mh / (sqrtf(vh) + a.eps);
        a.w[i] = w;
    }
    if (a.copy) a.copy[i] = (__bf16)w;
    if (a.copyT) a.copyT[(size_t)cc * a.rows + rr] = (__bf16)w;
}

__global__ void adam_kernel(AdamArgs a) {
    const size_t n = (size_t)a.rows * a.cols;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        adam_element(a, i);
}

// Every tensor of a batch in one grid-stride pass (element-wise identical to adam_kernel).
__global__ void adam_batch_kernel(AdamBatch b) {
    const size_t n = b.start[b.count];
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        int k = 0;
        while (k + 1 < b.count && i >= b.start[k + 1]) ++k;
        adam_element(b.t[k], i - b.start[k]);
    }
}

// Network inputs of a batch: X[b][0..D) = y, X[b][D] = SNR feature of sigma2[b], rest 0,
// as BF16 row-major (B x 16) and transposed (32 x B, rows 16..31 zero).  The SNR feature is
// (s - 7.5) / 7.5 with s = -10 log10(2 sigma2), the SNR in dB at unit energy per two dimensions.
__global__ void features_kernel(const float* y, const float* sigma2, int B, int D, __bf16* X, __bf16* Xt) {
    for (int b = blockIdx.x * blockDim.x + threadIdx.x; b < B; b += gridDim.x * blockDim.x) {
        // -10 log10(2 s2) = -(10 / log2(10)) (1 + log2 s2)
        const float snr_db = -3.0102999566398120f * (1.0f + __builtin_amdgcn_logf(sigma2[b]));
        for (int k = 0; k < 16; ++k) {
            float v = 0.0f;
            if (k < D) v = y[(size_t)b * D + k];
            else if (k == D) v = (snr_db - 7.5f) * (1.0f / 7.5f);
            const __bf16 q = (__bf16)v;
            X[(size_t)b * 16 + k] = q;
            Xt[(size_t)k * B + b] = q;
        }
        for (int k = 16; k < 32; ++k) Xt[(size_t)k * B + b] = (__bf16)0.0f;
    }
}

}  // namespace

hipError_t launch_gemm_nt(const GemmArgs& g, hipStream_t st) {
    if (g.M % 32 || g.N % 32 || g.K % 16 || g.splits < 1 || (g.K / g.splits) % 16 || g.K % g.splits)
        return hipErrorInvalidValue;
    const int waves = (g.M / 32) * (g.N / 32) * g.splits;
    const dim3 grid((waves + 3) / 4), block(256);
    if (g.A_lo && g.Bt_lo) hipLaunchKernelGGL((gemm_nt_kernel<true, true>), grid, block, 0, st, g);
    else if (g.A_lo) hipLaunchKernelGGL((gemm_nt_kernel<true, false>), grid, block, 0, st, g);
    else if (g.Bt_lo) hipLaunchKernelGGL((gemm_nt_kernel<false, true>), grid, block, 0, st, g);
    else hipLaunchKernelGGL((gemm_nt_kernel<false, false>), grid, block, 0, st, g);
    return hipGetLastError();
}

hipError_t launch_rowsum(const __bf16* X, const __bf16* Xlo, int rows, int cols, int ld, float* out, hipStream_t st) {
    hipLaunchKernelGGL(rowsum_kernel, dim3(rows), dim3(256), 0, st, X, Xlo, rows, cols, ld, out);
    return hipGetLastError();
}

hipError_t launch_reduce_splits(const float* part, int splits, size_t n, float* grad, hipStream_t st) {
    hipLaunchKernelGGL(reduce_splits_kernel, dim3(256), dim3(256), 0, st, part, splits, n, grad);
    return hipGetLastError();
}

hipError_t launch_adam_batch(const AdamBatch& b, hipStream_t st) {
    hipLaunchKernelGGL(adam_batch_kernel, dim3(256), dim3(256), 0, st, b);
    return hipGetLastError();
}

hipError_t launch_adam(const AdamArgs& a, hipStream_t st) {
    hipLaunchKernelGGL(adam_kernel, dim3(256), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_features(const float* y, const float* sigma2, int B, int D, __bf16* X, __bf16* Xt, hipStream_t st) {
    hipLaunchKernelGGL(features_kernel, dim3(256), dim3(256), 0, st, y, sigma2, B, D, X, Xt);
    return hipGetLastError();
}

}  // namespace dm
