// Tile loop and subset sums of the MFMA demapper for constellations of 32 to 256 points (one
// to eight 32-point tiles), with the tile count NT and the label-bit count m = 5 + log2(NT) fixed
// at compile time (shared by the single-constellation kernel and the batched kernel):
//   * the tile loop is fully unrolled: no per-tile guards and no pipelined MFMA of a tile past
//     the table;
//   * the first tile initialises the register-indexed sums (no zeroing per batch), and each
//     tile's 16-point total stays in a register of its own: label bits 5 and up are sums of
//     those totals, formed once per batch.
// The arithmetic (operand layout, exponents, label order) is that of mfma_body.hpp.
#pragma once
#include "mfma_body.hpp"

namespace dm {

constexpr int small_ilog2(int v) { return v <= 1 ? 0 : 1 + small_ilog2(v / 2); }

// Label bits of an NT-tile constellation.
template <int NT>
struct SmallBits {
    static constexpr int LB = small_ilog2(NT);  // carried by the tile index
    static constexpr int MB = 5 + LB;           // all label bits
};

// This wave's 32 symbols (operand fragments bfr) against tiles 0..NT-1 of the fragment table
// staged at lds_frag ([tile][s][lane] x 16 bytes): this lane half's subset sums S0 / S1 of every
// label bit and its total tot (bit 4 is the lane half; see mfma_finish).
template <typename T, int D, bool SPLIT, int NT>
__device__ __forceinline__ void mfma_small_sums(const uint4* lds_frag, int lane, const Frags<T, Slots<D, SPLIT>::S>& bfr,
                                                float (&S0)[SmallBits<NT>::MB], float (&S1)[SmallBits<NT>::MB],
                                                float& tot) {
    using V = typename Mma<T>::V;
    constexpr int S = Slots<D, SPLIT>::S;
    constexpr int LB = SmallBits<NT>::LB;
    const int h = lane >> 5;
    auto tile_mma = [&](int t) {
        const uint4* fp = lds_frag + t * S * 64 + lane;
        f32x16 acc = Mma<T>::run(__builtin_bit_cast(V, fp[0]), bfr.v[0]);
#pragma unroll
        for (int s = 1; s < S; ++s) acc = Mma<T>::run(__builtin_bit_cast(V, fp[s * 64]), bfr.v[s], acc);
        return acc;
    };
    // Tile t's MFMAs are issued before the exp2s of tile t - 1 (two alternating accumulators).
    float accA[16], tt[NT];
    f32x16 acc0 = tile_mma(0), acc1;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        if (t + 1 < NT) {
            if (t % 2 == 0) acc1 = tile_mma(t + 1);
            else acc0 = tile_mma(t + 1);
        }
        const f32x16& x = (t % 2 == 0) ? acc0 : acc1;
        float e[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) e[q] = hw_exp2(x[q]);
#pragma unroll
        for (int q = 0; q < 16; ++q) accA[q] = t == 0 ? e[q] : accA[q] + e[q];
        tt[t] = (((e[0] + e[1]) + (e[2] + e[3])) + ((e[4] + e[5]) + (e[6] + e[7]))) +
                (((e[8] + e[9]) + (e[10] + e[11])) + ((e[12] + e[13]) + (e[14] + e[15])));
        // One tile in flight at a time: the tile's exponentials are complete here and the next
        // tiles' LDS reads stay below (a memory clobber), so the compiler cannot issue every
        // tile's MFMAs up front (16 live accumulators per tile), which spills.
        asm volatile("" : "+v"(tt[t])::"memory");
    }
    // Bits 0-3 from the register-indexed sums, bit 4 the lane half, bits 5 and up from the tile
    // totals (tile index bit i = label bit 5 + i).
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
#pragma unroll
    for (int i = 0; i < LB; ++i) {
        float z = 0.0f, o = 0.0f;
        bool z0 = true, o0 = true;
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            if ((t >> i) & 1) {
                o = o0 ? tt[t] : o + tt[t];
                o0 = false;
            } else {
                z = z0 ? tt[t] : z + tt[t];
                z0 = false;
            }
        }
        S0[5 + i] = z;
        S1[5 + i] = o;
    }
}

// Far-subset pass of an NT-tile constellation's 32-symbol batch (both lane halves of every
// symbol call it; uniform per wave).  mask / near: the symbol's fix-up mask and near word from
// mfma_finish (deferred); y, c, K: the symbol and its block's exponent scale and offset.  A
// flagged bit whose symbol passed its near log-sum has a far subset whose terms all lie below
// the flag bound sh = m - 102, so the batch runs the tile loop again with the exponent offset
// lowered by sh: every far term is then kept to FP32 precision down to 2^-126, while near terms
// overflow to +inf -- harmlessly, since every register-indexed sum and tile total that makes up
// a far subset holds far terms only.  L = (sh + log2 S_far) - (near log-sum) with the sign of the
// far side, the same exponent arithmetic as every other LLR of the precision; the LLR is
// written, its GMI term added to g and the bit cleared from mask.  A far sum under 2^-95 (where
// flushed terms could matter) leaves its bit in mask for the fix-up queue, as do symbols
// without the near log-sum and the MI term.  When the pass has tried every flagged bit of a
// symbol, near is set to kNearNone: the bits left would fail the fix-up's far-only sum the same
// way (same shift, same bound), so the fix-up takes their two-pass sums at once.
template <typename T, int D, bool SPLIT, int NT>
__device__ __forceinline__ void mfma_small_far_pass(const uint4* lds_frag, int lane, const float (&y)[D], float c,
                                                    float K, bool bad, const BlockView& b, int64_t n, bool active,
                                                    int txl, uint32_t& near, uint32_t& mask, float& g) {
    constexpr int MB = SmallBits<NT>::MB;
    constexpr int S = Slots<D, SPLIT>::S;
    constexpr float sh = (float)(MB - 102);
    constexpr uint32_t kFarMask = (1u << (MB < kFarBits ? MB : kFarBits)) - 1u;
    const uint32_t far = (active && near != kNearNone) ? (mask & kFarMask) : 0u;
    if (__ballot(far != 0u) == 0ull) return;  // uniform per wave
    const int h = lane >> 5;
    bool bad2 = false;
    const Frags<T, S> bfr2 = build_symbol_frags<T, D, SPLIT>(y, c, K - sh, h, bad2);
    float S0[MB], S1[MB], tot;
    mfma_small_sums<T, D, SPLIT, NT>(lds_frag, lane, bfr2, S0, S1, tot);
    const bool bad_sym = half_or((uint32_t)(bad || bad2)) != 0;
    const float near_lse = __builtin_bit_cast(float, near);
    uint32_t done = 0u;
#pragma unroll
    for (int j = 0; j < (MB + 1) / 2; ++j) {
        // lane half h finishes bit 2j + h (the halves' partial sums meet in one swap)
        const float c0 = half_pair_sum(S0[2 * j], 2 * j + 1 < MB ? S0[2 * j + 1] : 0.0f);
        const float c1 = half_pair_sum(S1[2 * j], 2 * j + 1 < MB ? S1[2 * j + 1] : 0.0f);
        const int p = 2 * j + h;
        if (p < MB && ((far >> p) & 1u) && !bad_sym) {
            const int fb = (int)((mask >> (kFarShift + p)) & 1u);
            const float sf = fb ? c1 : c0;
            if (sf >= 0x1p-95f && sf < 3.0e38f) {
                const float lf = sh + hw_log2(sf);
                const float L = fb ? lf - near_lse : near_lse - lf;
                if (b.llr) b.llr[(size_t)n * MB + (MB - 1 - p)] = L * 0.69314718055994531f;
                if (b.tx) g += gmi_bit_term(L, (txl >> p) & 1);
                done |= 1u << p;
            }
        }
    }
    mask &= ~half_or(done);
    if (far != 0u && !bad_sym) near = kNearNone;
}

}  // namespace dm
