// Body of the exact soft demapper with the distance cross term on MFMA (gfx950, BF16/FP16 operands,
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
// label bits 0-3, the lane half is label bit 4 and the tile index gives bits 5 and up
// (bits 5-6: accB, 7-8: accC, 9 and up: per 512-label block sums).
// Per (symbol, point): one exp2 and two adds (accA[r] += e, T += e); see the FP32 kernel
// for the accumulation scheme, the underflow flag and the fix-up.
#pragma once
#include "device_common.hpp"

namespace dm {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(8 * sizeof(_Float16)))) _Float16 f16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;

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

// v_permlane32_swap of two registers: afterwards lane i < 32 holds (a[i], a[i+32]) and lane
// i + 32 holds (b[i], b[i+32]) in (r0, r1).  So r0 + r1 is a's two-half total in the lower half
// of the wave and b's in the upper half, without an LDS round trip.
__device__ __forceinline__ void swap_halves(uint32_t a, uint32_t b, uint32_t& r0, uint32_t& r1) {
    const auto r = __builtin_amdgcn_permlane32_swap(a, b, false, false);
    r0 = r[0];
    r1 = r[1];
}

__device__ __forceinline__ float half_pair_sum(float a, float b) {
    uint32_t r0, r1;
    swap_halves(__builtin_bit_cast(uint32_t, a), __builtin_bit_cast(uint32_t, b), r0, r1);
    return __builtin_bit_cast(float, r0) + __builtin_bit_cast(float, r1);
}

__device__ __forceinline__ uint32_t half_or(uint32_t a) {
    uint32_t r0, r1;
    swap_halves(a, a, r0, r1);
    return r0 | r1;
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

struct MfmaAcc {
    float accA[16], accB[4], accC[4], hi0[7], hi1[7];
    __device__ __forceinline__ void init() {
#pragma unroll
        for (int i = 0; i < 16; ++i) accA[i] = 0.0f;
#pragma unroll
        for (int i = 0; i < 4; ++i) accB[i] = accC[i] = 0.0f;
#pragma unroll
        for (int i = 0; i < 7; ++i) hi0[i] = hi1[i] = 0.0f;
    }
};

// Tiles the LDS copy of a cnt-tile chunk must span: the pipeline in mfma_tiles reads one
// tile past each 16-tile block (that read is never consumed).
constexpr int mfma_lds_tiles(int cnt) { return ((cnt + 15) / 16) * 16 + 1; }

// Tiles [0, cnt) of the fragment table staged at lds_frag, global tile index t0 + t (t0 a
// multiple of 16), against this wave's 32 symbols (operand fragments bfr).
template <typename T, int D, bool SPLIT>
__device__ __forceinline__ void mfma_tiles(const uint4* lds_frag, int lane, int t0, int cnt, int m,
                                           const Frags<T, Slots<D, SPLIT>::S>& bfr, MfmaAcc& A) {
    using V = typename Mma<T>::V;
    constexpr int S = Slots<D, SPLIT>::S;
    float (&accA)[16] = A.accA;
    float (&accB)[4] = A.accB;
    float (&accC)[4] = A.accC;
    float (&hi0)[7] = A.hi0;
    float (&hi1)[7] = A.hi1;
    // Software pipeline: the MFMAs of tile t+1 are issued before the exp2s of tile t.
    // Even tiles use acc0, odd tiles acc1 (no register copies); the next-tile MFMA is
    // unconditional, only the consumption is guarded.  Blocks of 16 tiles (512 labels) are
    // unrolled so that label bits 5-6 index accB and 7-8 accC, and tile t+1 is read at a
    // constant offset from the block's base address: the staged table must therefore extend
    // to tile roundup(cnt, 16) (mfma_lds_tiles), whose contents are never consumed.
    auto tile_mma = [&](int t) {
        const uint4* fp = lds_frag + (size_t)t * S * 64 + lane;
        f32x16 acc = Mma<T>::run(__builtin_bit_cast(V, fp[0]), bfr.v[0]);
#pragma unroll
        for (int s = 1; s < S; ++s) acc = Mma<T>::run(__builtin_bit_cast(V, fp[s * 64]), bfr.v[s], acc);
        return acc;
    };
    auto consume = [&](const f32x16& acc) {
        float e[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) e[r] = hw_exp2(acc[r]);
#pragma unroll
        for (int r = 0; r < 16; ++r) accA[r] += e[r];
        return (((e[0] + e[1]) + (e[2] + e[3])) + ((e[4] + e[5]) + (e[6] + e[7]))) +
               (((e[8] + e[9]) + (e[10] + e[11])) + ((e[12] + e[13]) + (e[14] + e[15])));
    };
    f32x16 acc0 = tile_mma(0), acc1;
    for (int b0 = 0; b0 < cnt; b0 += 16) {
        float bt = 0.0f;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            float gt = 0.0f;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int t = b0 + 4 * q + u;
                if (u % 2 == 0) {
                    acc1 = tile_mma(t + 1);
                    if (t < cnt) {
                        const float T16 = consume(acc0);
                        accB[u] += T16;
                        gt += T16;
                    }
                } else {
                    acc0 = tile_mma(t + 1);
                    if (t < cnt) {
                        const float T16 = consume(acc1);
                        accB[u] += T16;
                        gt += T16;
                    }
                }
            }
            accC[q] += gt;
            bt += gt;
        }
        const int blk = (t0 + b0) >> 4;  // label bits 9 and up
#pragma unroll
        for (int p = 9; p < 16; ++p) {
            if (p < m) {
                if ((blk >> (p - 9)) & 1) hi1[p - 9] += bt;
                else hi0[p - 9] += bt;
            }
        }
    }
}

// Per-half subset sums of every label bit from the tile-loop accumulators: S0[p] / S1[p] sum
// this lane half's points whose label bit p is 0 / 1, tot all of them.  Bits 0-3 index the
// 16 registers: their marginals share one pairwise tree (P: pairs over bit 0, Q: pairs of P
// over bit 1); bit 4 is the lane half; bits 5-6 and 7-8 index accB and accC; higher bits were
// summed per 512-label block.
__device__ __forceinline__ void mfma_subset_sums(const MfmaAcc& A, int h, float (&S0)[16], float (&S1)[16],
                                                 float& tot) {
    const float (&accA)[16] = A.accA;
    const float (&accB)[4] = A.accB;
    const float (&accC)[4] = A.accC;
    float P[8], Q[4];
#pragma unroll
    for (int q = 0; q < 8; ++q) P[q] = accA[2 * q] + accA[2 * q + 1];
#pragma unroll
    for (int u = 0; u < 4; ++u) Q[u] = P[2 * u] + P[2 * u + 1];
    S0[0] = ((accA[0] + accA[2]) + (accA[4] + accA[6])) + ((accA[8] + accA[10]) + (accA[12] + accA[14]));
    S1[0] = ((accA[1] + accA[3]) + (accA[5] + accA[7])) + ((accA[9] + accA[11]) + (accA[13] + accA[15]));
    S0[1] = (P[0] + P[2]) + (P[4] + P[6]);
    S1[1] = (P[1] + P[3]) + (P[5] + P[7]);
    S0[2] = Q[0] + Q[2];
    S1[2] = Q[1] + Q[3];
    S0[3] = Q[0] + Q[1];
    S1[3] = Q[2] + Q[3];
    tot = S0[3] + S1[3];
    S0[4] = h ? 0.0f : tot;
    S1[4] = h ? tot : 0.0f;
    S0[5] = accB[0] + accB[2];
    S1[5] = accB[1] + accB[3];
    S0[6] = accB[0] + accB[1];
    S1[6] = accB[2] + accB[3];
    S0[7] = accC[0] + accC[2];
    S1[7] = accC[1] + accC[3];
    S0[8] = accC[0] + accC[1];
    S1[8] = accC[2] + accC[3];
#pragma unroll
    for (int p = 9; p < 16; ++p) {
        S0[p] = A.hi0[p - 9];
        S1[p] = A.hi1[p - 9];
    }
}

// Combine the two lanes of each symbol, write LLRs, flag and queue underflowed bits and form
// the per-symbol GMI (both halves) and MI (half 0) terms, from this half's subset sums S0 / S1
// and total tot.  MB < 16: the constellation has exactly MB label bits (known at compile
// time); MB == 16: b.m bits.  txl is the symbol's transmitted label (0 without tx), loaded by
// the caller before the tile loop so that its latency is hidden.  With a non-null defer the
// flagged bits are not queued: *defer receives the symbol's fix-up mask (both halves) and
// defer_near its FixEntry.near word, for the caller to resolve or queue.
template <typename T, int D, bool SPLIT, int MB>
__device__ __forceinline__ void mfma_finish(const BlockView& b, const Sinks& k, const uint16_t* pv,
                                            const Frags<T, Slots<D, SPLIT>::S>& bfr, const float (&S0)[MB],
                                            const float (&S1)[MB], float tot, int64_t n, bool active, bool bad,
                                            int txl, int lane, float& g, float& mi, uint32_t* defer = nullptr,
                                            uint32_t* defer_near = nullptr, const float* ttx_direct = nullptr) {
    using V = typename Mma<T>::V;
    constexpr int S = Slots<D, SPLIT>::S;
    constexpr int NJ = (MB + 1) / 2;
    const int h = lane >> 5;
    const int m = MB < 16 ? MB : b.m;
    // Combine with the partner lane: half h finishes bit 2j + h of every pair (2j, 2j+1) as
    // its own partial sum plus the partner's.
    float c0[NJ], c1[NJ];
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        if (2 * j < m) {
            const float a0 = S0[2 * j], a1 = S1[2 * j];
            const float b0 = 2 * j + 1 < MB ? S0[2 * j + 1] : 0.0f, b1 = 2 * j + 1 < MB ? S1[2 * j + 1] : 0.0f;
            c0[j] = half_pair_sum(a0, b0);
            c1[j] = half_pair_sum(a1, b1);
        }
    }
    const bool bad_sym = half_or((uint32_t)bad) != 0;
    const float stot = half_pair_sum(tot, tot);

    g = 0.0f;
    uint32_t mask = 0;
    // Lane half h finishes bits p = 2j + h: the same j for both halves keeps the control flow
    // uniform, so every bit is processed once per wave.  The loop has no branches: a bit whose
    // sums are out of range gets a placeholder LLR, which the fix-up overwrites, and no GMI
    // term.  The range test runs on the bit patterns (the sums are non-negative, so unsigned
    // order is float order, and a NaN compares above the upper bound).
    const uint32_t lo_u = __builtin_bit_cast(uint32_t, b.flag_thresh);
    const uint32_t hi_u = __builtin_bit_cast(uint32_t, 3.0e38f);
    // An opaque copy of h: the lane tests below are then formed per batch (one compare each)
    // instead of being hoisted out of the symbol loop as per-bit lane masks, which spilled.
    int hv = h;
    asm volatile("" : "+v"(hv));
    uint32_t flagged = 0;
    float Lv[NJ];
    // the symbol's total, shared by every bit's GMI term (s0 + s1 = stot)
    const int es = __builtin_amdgcn_frexp_expf(stot);
    const float ls = hw_log2(__builtin_amdgcn_frexp_mantf(stot));
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        if (2 * j < m) {
            const int p = 2 * j + hv;
            const bool valid = p < m;  // false only in half 1 for the top bit of an odd m
            const float s0 = c0[j], s1 = c1[j];
            const uint32_t u0 = __builtin_bit_cast(uint32_t, s0), u1 = __builtin_bit_cast(uint32_t, s1);
            const bool ok = !bad_sym && min(u0, u1) >= lo_u && max(u0, u1) < hi_u;
            float gb;
            Lv[j] = llr_gmi(s0, s1, (txl >> p) & 1, es, ls, gb) * 0.69314718055994531f;
            g += (valid && ok) ? gb : 0.0f;
            flagged |= (valid && !ok) ? 1u << p : 0u;
        }
    }
    // Stores after the loop, at constant offsets from one column pointer (bit 2j + h is
    // column m - 1 - 2j - h), so that no store's registers are overwritten while it is in flight.
    if (b.llr && active) {
        float* col = b.llr + (size_t)n * m + (m - 1 - hv);
#pragma unroll
        for (int j = 0; j < NJ; ++j)
            if (2 * j < m && 2 * j + hv < m) col[-2 * j] = Lv[j];
    }
    if (flagged) {  // rare: the GMI-only shortcut, else the exact fix-up
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
            if (2 * j < m) {
                const int p = 2 * j + h;
                const float s0 = c0[j], s1 = c1[j];
                if ((flagged >> p) & 1) {
                    const int bit = (txl >> p) & 1;
                    if (!bad_sym && !b.want_llr && fmaxf(s0, s1) >= b.near_thresh && fmaxf(s0, s1) < 3.0e38f &&
                        (bit ? s1 > s0 : s0 > s1))
                        g += 1.0f;
                    else if constexpr (MB <= 8)
                        mask |= flag_bits(p, s0, s1);  // the row fix-up of M <= 256 uses the far side
                    else
                        mask |= 1u << p;
                }
            }
        }
    }
    // MI term: the exponent of the transmitted point comes from the same MFMA arithmetic
    // as the sum (so the rounding of beta and of the cross term cancels): lane l feeds row
    // l%32 with the point-side vector of its own symbol's transmitted label; the diagonal
    // element (l%32, l%32) sits in register 4*(j>>3) + (j&3) of the lane half (j>>2)&1.
    mi = 0.0f;
    if (b.tx && ttx_direct) {
        // the caller's FP32 exponent of the transmitted point, K - c ||y - x_tx||^2 from the
        // direct differences: it differs from that point's MFMA exponent inside stot by the
        // operands' rounding (~1e-5 in log2 units for the split precisions), not by a bias
        if (h == 0) {
            if (!bad_sym && stot >= b.flag_thresh && stot < 3.0e38f) {
                const int e = __builtin_amdgcn_frexp_expf(stot);
                const float mant = __builtin_amdgcn_frexp_mantf(stot);
                mi = ((float)(m - e) + *ttx_direct) - hw_log2(mant);
            } else {
                mask |= kMiFlag;
            }
        }
    } else if (b.tx) {
        const uint16_t* pr = pv + (size_t)txl * (16 * S) + 8 * h;
        f32x16 dg = Mma<T>::run(__builtin_bit_cast(V, *(const uint4*)pr), bfr.v[0]);
#pragma unroll
        for (int s2 = 1; s2 < S; ++s2)
            dg = Mma<T>::run(__builtin_bit_cast(V, *(const uint4*)(pr + 16 * s2)), bfr.v[s2], dg);
        const int j = lane & 31;
        int rd = 4 * (j >> 3) + (j & 3);
        asm volatile("" : "+v"(rd));  // keeps the lane masks below from being hoisted out of the loop
        float v;
        if constexpr (MB <= 8) {
            // dg[rd] by a four-level tree of bit selects (all-ones masks from the bits of rd): no
            // serial compare chain, and no run-time register index for the compiler to form.
            // The constellations of up to 256 points have the registers for it; the larger ones,
            // at the 128-register cap, keep the compare chain below.
            // (each element is copied to a scalar before the bit cast: this compiler casts
            // element 0 for a bit cast applied to an element of a vector-typed value)
            uint32_t w[16];
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const float f = dg[r];
                w[r] = __builtin_bit_cast(uint32_t, f);
            }
#pragma unroll
            for (int lvl = 0; lvl < 4; ++lvl) {
                const uint32_t pick = 0u - (((uint32_t)rd >> lvl) & 1u);  // 0 or all ones
#pragma unroll
                for (int i = 0; i < (8 >> lvl); ++i) w[i] = (w[2 * i + 1] & pick) | (w[2 * i] & ~pick);
            }
            v = __builtin_bit_cast(float, w[0]);
        } else {
            v = dg[0];
#pragma unroll
            for (int r = 1; r < 16; ++r) v = (rd == r) ? dg[r] : v;
        }
        // The lane half (j >> 2) & 1 holds the diagonal element; after the swap it is r1 if
        // that half is the upper one, else r0, in both halves.
        uint32_t v0, v1;
        swap_halves(__builtin_bit_cast(uint32_t, v), __builtin_bit_cast(uint32_t, v), v0, v1);
        const float ttx = __builtin_bit_cast(float, ((j >> 2) & 1) ? v1 : v0);
        if (h == 0) {
            if (!bad_sym && stot >= b.flag_thresh && stot < 3.0e38f) {
                const int e = __builtin_amdgcn_frexp_expf(stot);
                const float mant = __builtin_amdgcn_frexp_mantf(stot);
                mi = ((float)(m - e) + ttx) - hw_log2(mant);
            } else {
                mask |= kMiFlag;
            }
        }
    }
    mask = half_or(mask);
    if (defer) {
        *defer = mask;
        *defer_near = near_word(stot, m, bad_sym);
        return;
    }
    if (mask && active && h == 0) {
        double gc = 0.0, mc = 0.0;
        queue_or_fix<D>(b, k, (uint32_t)n, mask, near_word(stot, m, bad_sym), gc, mc);
        g += (float)gc;
        mi += (float)mc;
    }
}


// Subset sums of the first MB label bits and mfma_finish with MB bits known at compile time
// (MB == 16: b.m bits at run time).
template <typename T, int D, bool SPLIT, int MB>
__device__ __forceinline__ void mfma_epilogue_m(const BlockView& b, const Sinks& k, const uint16_t* pv,
                                                const Frags<T, Slots<D, SPLIT>::S>& bfr, const MfmaAcc& A,
                                                int64_t n, bool active, bool bad, int txl, int lane, float& g,
                                                float& mi) {
    float S0a[16], S1a[16], tot;
    mfma_subset_sums(A, lane >> 5, S0a, S1a, tot);
    float S0[MB], S1[MB];
#pragma unroll
    for (int p = 0; p < MB; ++p) {
        S0[p] = S0a[p];
        S1[p] = S1a[p];
    }
    mfma_finish<T, D, SPLIT, MB>(b, k, pv, bfr, S0, S1, tot, n, active, bad, txl, lane, g, mi);
}

// The generic epilogue: subset sums from the accumulators, then mfma_finish over b.m bits; the
// constellations of 512 to 4096 points (m = 9..12) take epilogues with m fixed at compile time
// (no per-bit guards), the branch on m being uniform over the launch.
template <typename T, int D, bool SPLIT>
__device__ __forceinline__ void mfma_epilogue(const BlockView& b, const Sinks& k, const uint16_t* pv,
                                              const Frags<T, Slots<D, SPLIT>::S>& bfr, const MfmaAcc& A,
                                              int64_t n, bool active, bool bad, int txl, int lane, float& g,
                                              float& mi) {
    switch (b.m) {
        case 9: mfma_epilogue_m<T, D, SPLIT, 9>(b, k, pv, bfr, A, n, active, bad, txl, lane, g, mi); break;
        case 10: mfma_epilogue_m<T, D, SPLIT, 10>(b, k, pv, bfr, A, n, active, bad, txl, lane, g, mi); break;
        case 11: mfma_epilogue_m<T, D, SPLIT, 11>(b, k, pv, bfr, A, n, active, bad, txl, lane, g, mi); break;
        case 12: mfma_epilogue_m<T, D, SPLIT, 12>(b, k, pv, bfr, A, n, active, bad, txl, lane, g, mi); break;
        default: mfma_epilogue_m<T, D, SPLIT, 16>(b, k, pv, bfr, A, n, active, bad, txl, lane, g, mi);
    }
}

}  // namespace dm
