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

}  // namespace dm
