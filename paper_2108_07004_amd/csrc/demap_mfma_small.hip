// Exact soft demapper for constellations of 32 to 256 points (one to eight 32-point tiles) with
// the distance cross term on MFMA (gfx950): the multi-SNR launch over one constellation with the
// tile count fixed at compile time (tile loop and subset sums in mfma_small.hpp, epilogue in
// mfma_body.hpp).  The whole operand table (at most 8 tiles x 2 MFMAs x 1 KiB), the FP32 points
// (at most 8 KiB) and the row-to-label map are staged in LDS once per block, so that the
// transmitted label and its point, read once per batch, cost LDS rather than global-memory
// latency.  With split FP16 operands the MI term takes the transmitted point's exponent from the
// direct FP32 differences (a few VALU instructions) instead of a diagonal MFMA product and a
// register select; the other precisions keep the diagonal product (their per-label operand
// rows are staged too).
#include <type_traits>

#include "device_common.hpp"
#include "kernels.hpp"
#include "mfma_body.hpp"
#include "mfma_small.hpp"

namespace dm {

namespace {

constexpr int kThreads = 1024;  // 16 waves; one block per CU (128 VGPRs per lane)
constexpr int kWaves = kThreads / 64;

template <typename T, int D, bool SPLIT, int NT>
__global__ __launch_bounds__(kThreads) void demap_mfma_small_kernel(const LaunchArgs a, const uint4* __restrict__ frag,
                                                                    const uint16_t* __restrict__ pv) {
    constexpr int S = Slots<D, SPLIT>::S;
    constexpr int MB = SmallBits<NT>::MB;  // label bits of the constellation
    __shared__ uint4 lds_frag[NT * S * 64];     // [tile][s][lane] x 16 bytes
    __shared__ float lds_tab[NT * 32 * D];      // FP32 points in label order
    // the transmitted point's MI exponent from FP32 differences only with split FP16 operands
    constexpr bool kDirectTx = SPLIT && std::is_same<T, _Float16>::value;
    __shared__ uint4 lds_pv[kDirectTx ? 1 : NT * 32 * 2 * S];  // [label][16 S halves]
    __shared__ uint16_t lds_r2l[NT * 32];       // row -> label
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int h = lane >> 5;
    const int wave = tid >> 6;
    const int wave_slot = (blockIdx.x * kWaves + wave) % kAccSlots;
    const Sinks& k = a.sinks;
    for (int i = tid; i < NT * S * 64; i += kThreads) lds_frag[i] = frag[i];
    for (int i = tid; i < NT * 32 * D; i += kThreads) lds_tab[i] = a.table[i];
    if constexpr (!kDirectTx)
        for (int i = tid; i < NT * 32 * 2 * S; i += kThreads) lds_pv[i] = reinterpret_cast<const uint4*>(pv)[i];
    for (int i = tid; i < NT * 32; i += kThreads) lds_r2l[i] = a.row2label[i];
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
    int s_idx = (int)(blockIdx.x / blks_per_snr);
    int64_t r = blockIdx.x - (int64_t)s_idx * blks_per_snr;
    // The received symbols and transmitted rows of the next batch are loaded one batch ahead:
    // their latency overlaps the current batch's tile loop and epilogue.
    const int sub = wave * 32 + (lane & 31);
    auto fetch = [&](int s, int64_t rr, float (&yy)[D], uint32_t& row) {
        const int64_t n = rr * sym_per_blk + sub;
        const bool act = n < a.N;
        const float* yrow = a.snr[s].y + (size_t)(act ? n : 0) * D;
#pragma unroll
        for (int d = 0; d < D; ++d) yy[d] = yrow[d];
        row = (a.tx && act) ? (uint32_t)a.tx[n] : 0u;
    };
    float y_nx[D];
    uint32_t row_nx = 0;
    if ((int64_t)blockIdx.x < total) fetch(s_idx, r, y_nx, row_nx);
    for (int64_t bt = blockIdx.x; bt < total; bt += gridDim.x) {
        const int64_t n = r * sym_per_blk + sub;
        if (s_idx != cur) {
            if (cur >= 0 && k.acc) flush();
            gsum = msum = 0.0;
            cur = s_idx;
        }
        const bool active = n < a.N;
        const BlockView b = view_sym(a, s_idx, n, active);
        float y[D];
#pragma unroll
        for (int d = 0; d < D; ++d) y[d] = active ? y_nx[d] : 0.0f;
        uint32_t row = row_nx;
        // next batch: advance (s_idx, r) and issue its loads
        r += gridDim.x;
        while (r >= blks_per_snr) {
            r -= blks_per_snr;
            ++s_idx;
        }
        if (bt + gridDim.x < total) fetch(s_idx, r, y_nx, row_nx);
        int txl = 0;
        if (b.tx && active) {
            if (row >= (uint32_t)b.M) {  // out-of-range row: clamped and reported
                if (k.bad_tx) atomicOr(k.bad_tx, 1u);
                row = 0;
            }
            txl = (int)lds_r2l[row];
        }
        bool bad = false;
        const Frags<T, S> bfr = build_symbol_frags<T, D, SPLIT>(y, b.c, b.K, h, bad);

        float S0[MB], S1[MB], tot;
        mfma_small_sums<T, D, SPLIT, NT>(lds_frag, lane, bfr, S0, S1, tot);
        // The MI term's exponent of the transmitted point: with split FP16 operands from the
        // direct FP32 differences (the MFMA exponents carry ~1e-6 of rounding, which then stays
        // in the MI term instead of cancelling); with the coarser BF16 split and the plain
        // operands from the same MFMA arithmetic as the sum, so that the transmitted point's own
        // rounding cancels (with BF16 splits the direct form was 1.2e-4 bit off in MI on
        // DP-16QAM at high SNR).
        const float ttx = fmaf(-b.c, sqdist<D>(y, lds_tab + txl * D), b.K);
        float g, mi;
        uint32_t mask, near;
        mfma_finish<T, D, SPLIT, MB>(b, k, reinterpret_cast<const uint16_t*>(lds_pv), bfr, S0, S1, tot, n, active, bad,
                                     txl, lane, g, mi, &mask, &near, kDirectTx ? &ttx : nullptr);
        // far subsets of flagged bits resolved in the wave (at high SNR nearly every batch has
        // some; each would otherwise be a queue entry and a recomputation from the queue)
        mfma_small_far_pass<T, D, SPLIT, NT>(lds_frag, lane, y, b.c, b.K, bad, b, n, active, txl, near, mask, g);
        if (mask && active && h == 0) {
            double gc = 0.0, mc = 0.0;
            queue_or_fix<D>(b, k, (uint32_t)n, mask, near, gc, mc);
            g += (float)gc;
            mi += (float)mc;
        }
        if (k.acc && active) {
            gsum += (double)g;
            msum += (double)mi;
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
