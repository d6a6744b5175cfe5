// Exact soft demapper for constellations of 32 to 256 points (one to eight 32-point tiles) with
// the distance cross term on MFMA (gfx950).  The arithmetic is that of demap_mfma.hip
// (mfma_body.hpp: operand layout, exponents, LLR / GMI / MI epilogue); what differs is that the
// tile count NT and the number of label bits m = 5 + log2(NT) are compile-time constants:
//   * the tile loop is fully unrolled: no per-tile guards and no pipelined MFMA of a tile past
//     the table (the generic loop runs 16-tile blocks, so at M = 256 half of its MFMAs and
//     their serialised waits would be spent on tiles that do not exist);
//   * the first tile initialises the label-bit accumulators (no zeroing per batch), and each
//     tile's 16-point total stays in a register of its own: label bits 5 and up are sums of
//     those totals, formed once per batch;
//   * the epilogue handles exactly m bits (no runtime bit guards).
// The whole operand table (at most 8 tiles x 2 MFMAs x 1 KiB) is staged in LDS once per block.
#include "device_common.hpp"
#include "kernels.hpp"
#include "mfma_body.hpp"

namespace dm {

namespace {

constexpr int kThreads = 1024;  // 16 waves; one block per CU (128 VGPRs per lane)
constexpr int kWaves = kThreads / 64;

constexpr int ilog2(int v) { return v <= 1 ? 0 : 1 + ilog2(v / 2); }

template <typename T, int D, bool SPLIT, int NT>
__global__ __launch_bounds__(kThreads) void demap_mfma_small_kernel(const LaunchArgs a, const uint4* __restrict__ frag,
                                                                    const uint16_t* __restrict__ pv) {
    using V = typename Mma<T>::V;
    constexpr int S = Slots<D, SPLIT>::S;
    constexpr int LB = ilog2(NT);  // label bits carried by the tile index
    constexpr int MB = 5 + LB;     // label bits of the constellation
    __shared__ uint4 lds_frag[NT * S * 64];  // [tile][s][lane] x 16 bytes
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int h = lane >> 5;
    const int wave = tid >> 6;
    const int wave_slot = (blockIdx.x * kWaves + wave) % kAccSlots;
    const Sinks& k = a.sinks;
    for (int i = tid; i < NT * S * 64; i += kThreads) lds_frag[i] = frag[i];
    __syncthreads();

    const int64_t sym_per_blk = (int64_t)kWaves * 32;
    const int64_t blks_per_snr = (a.N + sym_per_blk - 1) / sym_per_blk;
    const int64_t total = blks_per_snr * a.n_snr;
    double gsum = 0.0, msum = 0.0;
    int cur = -1;
    auto flush = [&]() {
        const double gw = wave_sum(gsum), mw = wave_sum(msum);
        if (lane == 0) {
            acc_add(k.acc, cur, wave_slot, 0, gw);
            acc_add(k.acc, cur, wave_slot, 1, mw);
        }
    };
    auto tile_mma = [&](int t, const Frags<T, S>& bfr) {
        const uint4* fp = lds_frag + t * S * 64 + lane;
        f32x16 acc = Mma<T>::run(__builtin_bit_cast(V, fp[0]), bfr.v[0]);
#pragma unroll
        for (int s = 1; s < S; ++s) acc = Mma<T>::run(__builtin_bit_cast(V, fp[s * 64]), bfr.v[s], acc);
        return acc;
    };
    int s_idx = (int)(blockIdx.x / blks_per_snr);
    int64_t r = blockIdx.x - (int64_t)s_idx * blks_per_snr;
    for (int64_t bt = blockIdx.x; bt < total; bt += gridDim.x) {
        const int64_t n = r * sym_per_blk + wave * 32 + (lane & 31);
        if (s_idx != cur) {
            if (cur >= 0 && k.acc) flush();
            gsum = msum = 0.0;
            cur = s_idx;
        }
        const bool active = n < a.N;
        const BlockView b = view_sym(a, s_idx, n, active);
        const float* yrow = b.y + (size_t)(active ? n : 0) * D;
        float y[D];
#pragma unroll
        for (int d = 0; d < D; ++d) {
            const float v = yrow[d];
            y[d] = active ? v : 0.0f;
        }
        bool bad = false;
        const Frags<T, S> bfr = build_symbol_frags<T, D, SPLIT>(y, b.c, b.K, h, bad);
        const int txl = (b.tx && active) ? tx_label(b, k, n) : 0;

        // Tile t's MFMAs are issued before the exp2s of tile t - 1 (two alternating accumulators).
        float accA[16], tt[NT];
        f32x16 acc0 = tile_mma(0, bfr), acc1;
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            if (t + 1 < NT) {
                if (t % 2 == 0) acc1 = tile_mma(t + 1, bfr);
                else acc0 = tile_mma(t + 1, bfr);
            }
            const f32x16& x = (t % 2 == 0) ? acc0 : acc1;
            float e[16];
#pragma unroll
            for (int q = 0; q < 16; ++q) e[q] = hw_exp2(x[q]);
#pragma unroll
            for (int q = 0; q < 16; ++q) accA[q] = t == 0 ? e[q] : accA[q] + e[q];
            tt[t] = (((e[0] + e[1]) + (e[2] + e[3])) + ((e[4] + e[5]) + (e[6] + e[7]))) +
                    (((e[8] + e[9]) + (e[10] + e[11])) + ((e[12] + e[13]) + (e[14] + e[15])));
        }
        // Subset sums of this lane half: bits 0-3 from the register-indexed sums, bit 4 the lane
        // half, bits 5 and up from the tile totals (tile index bit i = label bit 5 + i).
        float S0[MB], S1[MB];
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
        const float tot = S0[3] + S1[3];
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
        float g, mi;
        mfma_finish<T, D, SPLIT, MB>(b, k, pv, bfr, S0, S1, tot, n, active, bad, txl, lane, g, mi);
        if (k.acc && active) {
            gsum += (double)g;
            msum += (double)mi;
        }
        r += gridDim.x;
        while (r >= blks_per_snr) {
            r -= blks_per_snr;
            ++s_idx;
        }
    }
    if (cur >= 0 && k.acc) flush();
}

template <typename T, int D, bool SPLIT>
hipError_t launch_nt(const LaunchArgs& a, const void* frag, const void* pv, int grid, hipStream_t st) {
    const uint4* f = (const uint4*)frag;
    const uint16_t* p = (const uint16_t*)pv;
    switch (a.M) {
        case 32: hipLaunchKernelGGL((demap_mfma_small_kernel<T, D, SPLIT, 1>), dim3(grid), dim3(kThreads), 0, st, a, f, p); break;
        case 64: hipLaunchKernelGGL((demap_mfma_small_kernel<T, D, SPLIT, 2>), dim3(grid), dim3(kThreads), 0, st, a, f, p); break;
        case 128: hipLaunchKernelGGL((demap_mfma_small_kernel<T, D, SPLIT, 4>), dim3(grid), dim3(kThreads), 0, st, a, f, p); break;
        case 256: hipLaunchKernelGGL((demap_mfma_small_kernel<T, D, SPLIT, 8>), dim3(grid), dim3(kThreads), 0, st, a, f, p); break;
        default: return hipErrorNotSupported;
    }
    return hipGetLastError();
}

template <typename T, bool SPLIT>
hipError_t launch_d(const LaunchArgs& a, const void* frag, const void* pv, int grid, hipStream_t st) {
    switch (a.D) {
        case 2: return launch_nt<T, 2, SPLIT>(a, frag, pv, grid, st);
        case 4: return launch_nt<T, 4, SPLIT>(a, frag, pv, grid, st);
        case 8: return launch_nt<T, 8, SPLIT>(a, frag, pv, grid, st);
        default: return hipErrorNotSupported;
    }
}

}  // namespace

bool mfma_small_supported(int M, int D) { return M >= 32 && M <= 256 && (D == 2 || D == 4 || D == 8); }

hipError_t launch_demap_mfma_small(const LaunchArgs& a, int prec, const void* frag, const void* pv, int grid,
                                   hipStream_t st) {
    if (!mfma_small_supported(a.M, a.D)) return hipErrorNotSupported;
    switch (prec) {
        case 1: return launch_d<__bf16, false>(a, frag, pv, grid, st);
        case 2: return launch_d<_Float16, false>(a, frag, pv, grid, st);
        case 3: return launch_d<__bf16, true>(a, frag, pv, grid, st);
        case 4: return launch_d<_Float16, true>(a, frag, pv, grid, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace dm
