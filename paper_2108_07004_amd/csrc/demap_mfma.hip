// Exact soft demapper with the distance cross term on MFMA (gfx950, BF16/FP16 operands,
// FP32 accumulation), hi/lo split variants, and the same log-sum-exp/GMI epilogue.
//
// For a received symbol y and a point x_j the kernel needs the exponent
//     t_j = K - c ||y - x_j||^2 = (K - c||y||^2) + 2c y.x_j - c||x_j||^2,   c = log2(e)/(2 sigma2).
// Each term is a K-slot product of a symbol-side vector and a point-side vector:
//   plain:  symbol [2cy (D), c, beta]                        point [x (D), -||x||^2, 1]
//   split:  symbol [hi(2cy), lo(2cy), hi(2cy), hi c, lo c, hi c, hi beta, lo beta]
//           point  [hi(x),   hi(x),   lo(x),   -hi n, -hi n, -lo n, 1, 1]          (n = ||x||^2)
// with beta = K - c||y||^2 and hi(v) = round(v), lo(v) = round(v - hi(v)) in the operand type, so
// the split form keeps hi*hi + lo*hi + hi*lo of every product (~2x the operand mantissa).
// One v_mfma_f32_32x32x16 multiplies a 32-point tile (rows) by 32 symbols (columns).
// Point rows are ordered so that lane l of the 32x32 result holds, in its 16 registers, the
// labels 32t + 16*(l/32) + r (r = 0..15) of tile t for symbol l%32: register r indexes
// label bits 0-3, the lane half is label bit 4 and the tile index gives bits 5 and up.
// Per (symbol, point): one exp2 and two adds (accA[r] += e, T += e); see the FP32 kernel
// for the accumulation scheme, the underflow flag and the fix-up.
#include "device_common.hpp"
#include "kernels.hpp"

namespace dm {

namespace {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(8 * sizeof(_Float16)))) _Float16 f16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;

constexpr int kMfmaThreads = 1024;  // 16 waves share one LDS copy of the point table
constexpr int kMfmaLdsBytes = 131072;

template <typename T>
struct Mma;
template <>
struct Mma<__bf16> {
    using V = bf16x8;
    static __device__ __forceinline__ f32x16 run(V a, V b) {
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, f32x16{}, 0, 0, 0);
    }
    static __device__ __forceinline__ f32x16 run(V a, V b, f32x16 c) {
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
    }
    static constexpr float kMax = 3.0e38f;
};
template <>
struct Mma<_Float16> {
    using V = f16x8;
    static __device__ __forceinline__ f32x16 run(V a, V b) {
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, f32x16{}, 0, 0, 0);
    }
    static __device__ __forceinline__ f32x16 run(V a, V b, f32x16 c) {
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
    }
    static constexpr float kMax = 60000.0f;
};

// Symbol-side K-slot roles.
enum : int { kZero = 0, kYhi = 1, kYlo = 2, kChi = 3, kClo = 4, kBhi = 5, kBlo = 6 };

template <int D, bool SPLIT>
struct Slots {
    static constexpr int used = SPLIT ? 3 * D + 5 : D + 2;
    static constexpr int S = (used + 15) / 16;  // MFMAs per tile (K = 16 each)
    // role and dimension of symbol-side slot k
    static constexpr int role(int k) {
        if (!SPLIT) return k < D ? kYhi : k == D ? kChi : k == D + 1 ? kBhi : kZero;
        if (k < D) return kYhi;
        if (k < 2 * D) return kYlo;
        if (k < 3 * D) return kYhi;
        const int q = k - 3 * D;
        return q == 0 ? kChi : q == 1 ? kClo : q == 2 ? kChi : q == 3 ? kBhi : q == 4 ? kBlo : kZero;
    }
    static constexpr int dim(int k) { return k % D; }
};

// hi/lo split of an FP32 value.  The value is pinned in a register first: otherwise the
// compiler may round an unrounded product straight to FP16 (mixed-precision FMA) for one
// copy of hi and convert the FP32-rounded product for another, and near rounding ties the
// two copies differ by one ulp of hi, which the lo part then no longer compensates.
template <typename T>
__device__ __forceinline__ void split2(float v, T& hi, T& lo) {
    asm volatile("" : "+v"(v));
    hi = (T)v;
    lo = (T)(v - (float)hi);
}

template <typename T>
__device__ __forceinline__ T round_pinned(float v) {
    asm volatile("" : "+v"(v));
    return (T)v;
}

// Builds this lane's symbol-side operand fragments: MFMA s, lane half h, values v = 0..7
// cover slot k = 16 s + 8 h + v.
template <typename T, int S>
struct Frags {
    typename Mma<T>::V v[S];
};

template <typename T, int D, bool SPLIT>
__device__ __forceinline__ Frags<T, Slots<D, SPLIT>::S> build_symbol_frags(const float (&y)[D], float c, float K, int h,
                                                                           bool& bad) {
    using Sl = Slots<D, SPLIT>;
    Frags<T, Sl::S> bf;
    T yh[D], yl[D];
    float ysq = 0.0f, ymax = 0.0f;
#pragma unroll
    for (int d = 0; d < D; ++d) {
        const float v = 2.0f * c * y[d];
        ymax = fmaxf(ymax, fabsf(v));
        ysq = fmaf(y[d], y[d], ysq);
        if constexpr (SPLIT) split2<T>(v, yh[d], yl[d]);
        else {
            yh[d] = round_pinned<T>(v);
            yl[d] = (T)0.0f;
        }
    }
    const float beta = fmaf(-c, ysq, K);
    T chi, clo, bhi, blo;
    if constexpr (SPLIT) {
        split2<T>(c, chi, clo);
        split2<T>(beta, bhi, blo);
    } else {
        chi = round_pinned<T>(c);
        clo = (T)0.0f;
        bhi = round_pinned<T>(beta);
        blo = (T)0.0f;
    }
    bad = !(ymax < Mma<T>::kMax) || !(fabsf(beta) < Mma<T>::kMax);
#pragma unroll
    for (int s = 0; s < Sl::S; ++s) {
#pragma unroll
        for (int v = 0; v < 8; ++v) {
            T val[2];
#pragma unroll
            for (int hh = 0; hh < 2; ++hh) {
                const int k = 16 * s + 8 * hh + v;
                const int role = Sl::role(k);
                const int d = Sl::dim(k);
                T x = (T)0.0f;
                if (role == kYhi) x = yh[d];
                else if (role == kYlo) x = yl[d];
                else if (role == kChi) x = chi;
                else if (role == kClo) x = clo;
                else if (role == kBhi) x = bhi;
                else if (role == kBlo) x = blo;
                val[hh] = x;
            }
            bf.v[s][v] = h ? val[1] : val[0];
        }
    }
    return bf;
}

template <typename T, int D, bool SPLIT>
__global__ __launch_bounds__(kMfmaThreads) void demap_mfma_kernel(const LaunchArgs a, const uint4* __restrict__ frag,
                                                                  const uint16_t* __restrict__ pv) {
    using Sl = Slots<D, SPLIT>;
    using V = typename Mma<T>::V;
    constexpr int S = Sl::S;
    extern __shared__ uint4 lds_frag[];  // [tile][s][64 lanes] x 16 bytes
    const int M = a.M, m = a.m;
    const int ntiles = M >> 5;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int h = lane >> 5;
    const int wave = tid >> 6;
    constexpr int kWaves = kMfmaThreads / 64;
    const int chunk_tiles = min(ntiles, kMfmaLdsBytes / (S * 64 * 16));
    const int nchunks = (ntiles + chunk_tiles - 1) / chunk_tiles;
    const int wave_slot = (blockIdx.x * kWaves + wave) % kAccSlots;

    auto stage = [&](int t0, int cnt) {
        const uint4* src = frag + (size_t)t0 * S * 64;
        for (int i = tid; i < cnt * S * 64; i += kMfmaThreads) lds_frag[i] = src[i];
    };
    if (nchunks == 1) {
        stage(0, ntiles);
        __syncthreads();
    }

    // Block-level symbol tiles of kWaves * 32 symbols; all waves iterate together so
    // chunked staging can synchronise the block.
    const int64_t sym_per_blk = (int64_t)kWaves * 32;
    const int64_t blks_per_snr = (a.N + sym_per_blk - 1) / sym_per_blk;
    const int64_t total = blks_per_snr * a.n_snr;
    double gsum = 0.0, msum = 0.0;
    int cur = -1;
    for (int64_t bt = blockIdx.x; bt < total; bt += gridDim.x) {
        const int s_idx = (int)(bt / blks_per_snr);
        const int64_t n = (bt % blks_per_snr) * sym_per_blk + wave * 32 + (lane & 31);
        if (s_idx != cur) {
            if (cur >= 0 && a.acc && lane == 0) {
                acc_add(a.acc, cur, wave_slot, 0, gsum);
                acc_add(a.acc, cur, wave_slot, 1, msum);
            }
            gsum = msum = 0.0;
            cur = s_idx;
        }
        const SnrArg sa = a.snr[s_idx];
        const bool active = n < a.N;
        const float c = sa.c, K = a.K;
        float y[D];
#pragma unroll
        for (int d = 0; d < D; ++d) y[d] = active ? sa.y[(size_t)n * D + d] : 0.0f;
        bool bad = false;
        const Frags<T, S> bfr = build_symbol_frags<T, D, SPLIT>(y, c, K, h, bad);

        float accA[16], accB[4], hi0[9], hi1[9];
#pragma unroll
        for (int i = 0; i < 16; ++i) accA[i] = 0.0f;
#pragma unroll
        for (int i = 0; i < 4; ++i) accB[i] = 0.0f;
#pragma unroll
        for (int i = 0; i < 9; ++i) hi0[i] = hi1[i] = 0.0f;

        for (int ch = 0; ch < nchunks; ++ch) {
            const int t0 = ch * chunk_tiles;
            const int cnt = min(chunk_tiles, ntiles - t0);
            if (nchunks > 1) {
                __syncthreads();
                stage(t0, cnt);
                __syncthreads();
            }
            // Software pipeline: the MFMAs of tile t+1 are issued before the exp2s of tile t.
            auto tile_mma = [&](int t) {
                const uint4* fp = lds_frag + (size_t)t * S * 64 + lane;
                f32x16 acc = Mma<T>::run(__builtin_bit_cast(V, fp[0]), bfr.v[0]);
#pragma unroll
                for (int s = 1; s < S; ++s) acc = Mma<T>::run(__builtin_bit_cast(V, fp[s * 64]), bfr.v[s], acc);
                return acc;
            };
            f32x16 cur = tile_mma(0);
            for (int g0 = 0; g0 < cnt; g0 += 4) {  // groups of 4 tiles = 128 labels
                float gt = 0.0f;
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int t = g0 + u;
                    if (t < cnt) {
                        const f32x16 nxt = (t + 1 < cnt) ? tile_mma(t + 1) : cur;
                        float e[16];
#pragma unroll
                        for (int r = 0; r < 16; ++r) e[r] = hw_exp2(cur[r]);
#pragma unroll
                        for (int r = 0; r < 16; ++r) accA[r] += e[r];
                        const float T16 = (((e[0] + e[1]) + (e[2] + e[3])) + ((e[4] + e[5]) + (e[6] + e[7]))) +
                                          (((e[8] + e[9]) + (e[10] + e[11])) + ((e[12] + e[13]) + (e[14] + e[15])));
                        accB[u] += T16;
                        gt += T16;
                        cur = nxt;
                    }
                }
                const int grp = (t0 + g0) >> 2;  // label bits 7 and up
#pragma unroll
                for (int p = 7; p < 16; ++p) {
                    if (p < m) {
                        if ((grp >> (p - 7)) & 1) hi1[p - 7] += gt;
                        else hi0[p - 7] += gt;
                    }
                }
            }
        }

        // Per-half marginals, then combine the two lanes (l, l^32) of each symbol.
        float S0[16], S1[16];
        float tot = 0.0f;
#pragma unroll
        for (int r = 0; r < 16; ++r) tot += accA[r];
#pragma unroll
        for (int p = 0; p < 16; ++p) {
            float s0 = 0.0f, s1 = 0.0f;
            if (p < 4) {
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    if ((r >> p) & 1) s1 += accA[r];
                    else s0 += accA[r];
                }
            } else if (p == 4) {
                s0 = h ? 0.0f : tot;
                s1 = h ? tot : 0.0f;
            } else if (p < 7) {
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    if ((u >> (p - 5)) & 1) s1 += accB[u];
                    else s0 += accB[u];
                }
            } else {
                s0 = hi0[p - 7];
                s1 = hi1[p - 7];
            }
            S0[p] = s0;
            S1[p] = s1;
        }
#pragma unroll
        for (int p = 0; p < 16; ++p) {
            if (p < m) {
                S0[p] += __shfl_xor(S0[p], 32, 64);
                S1[p] += __shfl_xor(S1[p], 32, 64);
            }
        }
        const bool bad_sym = bad || __shfl_xor((int)bad, 32, 64);
        const float stot = S0[0] + S1[0];

        const int txl = (a.tx && active) ? tx_label(a, n) : 0;
        float g = 0.0f;
        uint32_t mask = 0;
        float* out = (sa.llr && active) ? sa.llr + (size_t)n * m : nullptr;
#pragma unroll
        for (int p = 0; p < 16; ++p) {
            if (p < m && (p & 1) == h) {
                const float s0 = S0[p], s1 = S1[p];
                const bool flagged = bad_sym || !(fminf(s0, s1) >= a.flag_thresh) || !(fmaxf(s0, s1) < 3.0e38f);
                const float L = log2_ratio(s1, s0);
                const int b = (txl >> p) & 1;
                if (!flagged) {
                    if (out) out[m - 1 - p] = L * 0.69314718055994531f;
                    g += gmi_bit_term(L, b);
                } else if (!bad_sym && !a.want_llr && fmaxf(s0, s1) >= a.near_thresh &&
                           fmaxf(s0, s1) < 3.0e38f && (b ? s1 > s0 : s0 > s1)) {
                    g += 1.0f;
                } else {
                    mask |= 1u << p;
                }
            }
        }
        // MI term: the exponent of the transmitted point comes from the same MFMA arithmetic
        // as the sum (so the rounding of beta and of the cross term cancels): lane l feeds row
        // l%32 with the point-side vector of its own symbol's transmitted label; the diagonal
        // element (l%32, l%32) sits in register 4*(j>>3) + (j&3) of the lane half (j>>2)&1.
        float mi = 0.0f;
        if (a.tx) {
            const uint16_t* pr = pv + (size_t)txl * (16 * S) + 8 * h;
            f32x16 dg = Mma<T>::run(__builtin_bit_cast(V, *(const uint4*)pr), bfr.v[0]);
#pragma unroll
            for (int s2 = 1; s2 < S; ++s2)
                dg = Mma<T>::run(__builtin_bit_cast(V, *(const uint4*)(pr + 16 * s2)), bfr.v[s2], dg);
            const int j = lane & 31;
            const int rd = 4 * (j >> 3) + (j & 3);
            float v = dg[0];
#pragma unroll
            for (int r = 1; r < 16; ++r) v = (rd == r) ? dg[r] : v;
            const float vo = __shfl_xor(v, 32, 64);
            const float ttx = (((j >> 2) & 1) == h) ? v : vo;
            if (h == 0) {
                if (!bad_sym && stot >= a.flag_thresh && stot < 3.0e38f) {
                    const int e = __builtin_amdgcn_frexp_expf(stot);
                    const float mant = __builtin_amdgcn_frexp_mantf(stot);
                    mi = ((float)(m - e) + ttx) - hw_log2(mant);
                } else {
                    mask |= kMiFlag;
                }
            }
        }
        mask |= (uint32_t)__shfl_xor((int)mask, 32, 64);
        bool inline_fix = false;
        if (mask && active && h == 0) {
            if (a.fix_pairs) atomicAdd(a.fix_pairs + s_idx, (uint32_t)__popc(mask & 0xFFFFu));
            const uint32_t slot = atomicAdd(a.queue_count, 1u);
            if (slot < a.queue_cap) a.queue[slot] = FixEntry{(uint32_t)n, (uint32_t)s_idx, mask, 0u};
            else inline_fix = true;  // queue full: recompute in place (slow, still exact)
        }
        if (inline_fix) {
            double gc = 0.0, mc = 0.0;
            fixup_one<D>(a, FixEntry{(uint32_t)n, (uint32_t)s_idx, mask, 0u}, gc, mc);
            g += (float)gc;
            mi += (float)mc;
        }
        if (a.acc) {
            gsum += wave_sum(active ? (double)g : 0.0);
            msum += wave_sum(active ? (double)mi : 0.0);
        }
    }
    if (cur >= 0 && a.acc && lane == 0) {
        acc_add(a.acc, cur, wave_slot, 0, gsum);
        acc_add(a.acc, cur, wave_slot, 1, msum);
    }
}

template <typename T, int D, bool SPLIT>
hipError_t launch_t(const LaunchArgs& a, const void* frag, const void* pv, int grid, hipStream_t st) {
    constexpr int S = Slots<D, SPLIT>::S;
    const int ntiles = a.M >> 5;
    const int chunk_tiles = std::min(ntiles, kMfmaLdsBytes / (S * 64 * 16));
    const size_t lds = (size_t)chunk_tiles * S * 64 * 16;
    auto kern = demap_mfma_kernel<T, D, SPLIT>;
    hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(grid), dim3(kMfmaThreads), lds, st, a, (const uint4*)frag, (const uint16_t*)pv);
    return hipGetLastError();
}

template <typename T, bool SPLIT>
hipError_t launch_d(const LaunchArgs& a, const void* frag, const void* pv, int grid, hipStream_t st) {
    switch (a.D) {
        case 1: return launch_t<T, 1, SPLIT>(a, frag, pv, grid, st);
        case 2: return launch_t<T, 2, SPLIT>(a, frag, pv, grid, st);
        case 3: return launch_t<T, 3, SPLIT>(a, frag, pv, grid, st);
        case 4: return launch_t<T, 4, SPLIT>(a, frag, pv, grid, st);
        case 5: return launch_t<T, 5, SPLIT>(a, frag, pv, grid, st);
        case 6: return launch_t<T, 6, SPLIT>(a, frag, pv, grid, st);
        case 7: return launch_t<T, 7, SPLIT>(a, frag, pv, grid, st);
        case 8: return launch_t<T, 8, SPLIT>(a, frag, pv, grid, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

int mfma_slots(int D, bool split) {
    const int used = split ? 3 * D + 5 : D + 2;
    return 16 * ((used + 15) / 16);
}

int mfma_block_symbols() { return (kMfmaThreads / 64) * 32; }

hipError_t launch_demap_mfma(const LaunchArgs& a, int prec, const void* frag, const void* pv, int grid, hipStream_t st) {
    switch (prec) {
        case 1: return launch_d<__bf16, false>(a, frag, pv, grid, st);
        case 2: return launch_d<_Float16, false>(a, frag, pv, grid, st);
        case 3: return launch_d<__bf16, true>(a, frag, pv, grid, st);
        case 4: return launch_d<_Float16, true>(a, frag, pv, grid, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace dm
