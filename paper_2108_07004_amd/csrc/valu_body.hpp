// Per-symbol body of the FP32 direct-difference demapper (one lane = one symbol).
//
// For every point j the lane forms e_j = 2^(K - c ||y - x_j||^2), c = log2(e)/(2 sigma2): the
// likelihood exp(-||y-x||^2/(2 sigma2)) rescaled by the fixed factor 2^K, so no running maximum
// is needed (e_j <= 2^K because ||y-x||^2 >= 0, and K = 123 - m keeps the sum of M terms below
// 2^123).  The per-bit subset sums S_p^0, S_p^1 come from accumulators indexed by the label's
// low bits (table in label order):
//   bits 0-3: accA[j & 15] (one add per point); group sum T over 16 points (one add);
//   bits 4-5: accB[(j >> 4) & 3] (one add per 16 points);
//   bits >= 6: the 64-point block sum added to the side given by (j >> 6).
// A subset sum under 2^(m-102) may have lost terms below FP32's normal range (v_exp_f32 flushes
// results under 2^-126); such (symbol, bit) pairs are queued for an exact recomputation.
#pragma once
#include "device_common.hpp"

namespace dm {

// Accumulators: accA[16] (label bits 0-3), accB[4] (bits 4-5), hi0/hi1[10] (bits 6-15).
#define DM_VALU_ACC_DECL \
    float accA[16], accB[4], hi0[10], hi1[10]; \
    _Pragma("unroll") for (int i_ = 0; i_ < 16; ++i_) accA[i_] = 0.0f; \
    _Pragma("unroll") for (int i_ = 0; i_ < 4; ++i_) accB[i_] = 0.0f; \
    _Pragma("unroll") for (int i_ = 0; i_ < 10; ++i_) hi0[i_] = hi1[i_] = 0.0f;

// Accumulate the points [c0, c0 + cnt) of the label-ordered table staged at `lds` (cnt a
// multiple of 16, c0 a multiple of 64).
template <int DP>
__device__ __forceinline__ void valu_accumulate(const float* lds, int c0, int cnt, const float (&y)[DP], float c,
                                                float K, int m, float (&accA)[16], float (&accB)[4],
                                                float (&hi0)[10], float (&hi1)[10]) {
    for (int b0 = 0; b0 < cnt; b0 += 64) {
        float bt = 0.0f;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (b0 + q * 16 < cnt) {
                const float* xg = lds + (size_t)(b0 + q * 16) * DP;
                float T = 0.0f;
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const float e = hw_exp2(fmaf(-c, sqdist<DP>(y, xg + r * DP), K));
                    accA[r] += e;
                    T += e;
                }
                accB[q] += T;
                bt += T;
            }
        }
        const int blk = (c0 + b0) >> 6;
#pragma unroll
        for (int p = 6; p < 16; ++p) {
            if (p < m) {
                const bool one = (blk >> (p - 6)) & 1;
                hi1[p - 6] += one ? bt : 0.0f;
                hi0[p - 6] += one ? 0.0f : bt;
            }
        }
    }
}

// Per-bit subset sums -> LLRs, flags, GMI and MI terms of one symbol; queues flagged bits.
template <int DP>
__device__ __forceinline__ void valu_epilogue(const BlockView& b, const Sinks& k, int64_t n, bool active,
                                              const float (&y)[DP], const float (&accA)[16], const float (&accB)[4],
                                              const float (&hi0)[10], const float (&hi1)[10], float& g, float& mi) {
    const int m = b.m;
    const int txl = (b.tx && active) ? tx_label(b, k, n) : 0;
    float stot = 0.0f;
#pragma unroll
    for (int r = 0; r < 16; ++r) stot += accA[r];
    g = 0.0f;
    mi = 0.0f;
    uint32_t mask = 0;
    float* out = (b.llr && active) ? b.llr + (size_t)n * m : nullptr;
#pragma unroll
    for (int p = 0; p < 16; ++p) {
        if (p >= m) break;
        float s0 = 0.0f, s1 = 0.0f;
        if (p < 4) {
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                if ((r >> p) & 1) s1 += accA[r];
                else s0 += accA[r];
            }
        } else if (p < 6) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if ((q >> (p - 4)) & 1) s1 += accB[q];
                else s0 += accB[q];
            }
        } else {
            s0 = hi0[p - 6];
            s1 = hi1[p - 6];
        }
        const bool flagged = !(fminf(s0, s1) >= b.flag_thresh);
        const float L = log2_ratio(s1, s0);
        const int bit = (txl >> p) & 1;
        if (!flagged) {
            if (out) out[m - 1 - p] = L * 0.69314718055994531f;
            g += gmi_bit_term(L, bit);
        } else if (!b.want_llr && fmaxf(s0, s1) >= b.near_thresh && (bit ? s1 > s0 : s0 > s1)) {
            g += 1.0f;  // |L| >= 60 with the transmitted bit on the near side: term is 1 in FP64
        } else {
            mask |= flag_bits(p, s0, s1);
        }
    }
    if (b.tx) {
        if (stot >= b.flag_thresh) {
            const float ttx = fmaf(-b.c, sqdist<DP>(y, b.table + (size_t)txl * DP), b.K);
            const int e = __builtin_amdgcn_frexp_expf(stot);
            const float mant = __builtin_amdgcn_frexp_mantf(stot);
            // m - log2(stot) + t_tx, with log2(stot) = e + log2(mant) split off exactly
            mi = ((float)(m - e) + ttx) - hw_log2(mant);
        } else {
            mask |= kMiFlag;
        }
    }
    if (mask && active) {
        double gc = 0.0, mc = 0.0;
        queue_or_fix<DP>(b, k, (uint32_t)n, mask, near_word(stot, m, false), gc, mc);
        g += (float)gc;
        mi += (float)mc;
    }
}

}  // namespace dm
