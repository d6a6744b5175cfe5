// Exact soft demapper with the distance cross term on MFMA (gfx950): the multi-SNR launch over
// one constellation.  The per-tile arithmetic and the epilogue are in mfma_body.hpp.
#include "device_common.hpp"
#include "kernels.hpp"
#include "mfma_body.hpp"

namespace dm {

namespace {

constexpr int kMfmaThreads = 1024;  // 16 waves share one LDS copy of the point table
constexpr int kMfmaLdsBytes = 131072;

template <typename T, int D, bool SPLIT>
__global__ __launch_bounds__(kMfmaThreads) void demap_mfma_kernel(const LaunchArgs a, const uint4* __restrict__ frag,
                                                                  const uint16_t* __restrict__ pv) {
    constexpr int S = Slots<D, SPLIT>::S;
    extern __shared__ uint4 lds_frag[];  // [tile][s][64 lanes] x 16 bytes
    const int ntiles = a.M >> 5;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int h = lane >> 5;
    const int wave = tid >> 6;
    constexpr int kWaves = kMfmaThreads / 64;
    const int chunk_tiles = min(ntiles, kMfmaLdsBytes / (S * 64 * 16));
    const int nchunks = (ntiles + chunk_tiles - 1) / chunk_tiles;
    const int wave_slot = (blockIdx.x * kWaves + wave) % kAccSlots;
    const Sinks& k = a.sinks;

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
    // GMI / MI terms accumulate per lane in FP64 (fixed order: the blocks' symbol tiles are
    // assigned statically) and are summed over the wave only when the SNR point changes.
    double gsum = 0.0, msum = 0.0;
    int cur = -1;
    auto flush = [&]() {
        const double gw = wave_sum(gsum), mw = wave_sum(msum);
        if (lane == 0) {
            acc_add(k.acc, cur, wave_slot, 0, gw);
            acc_add(k.acc, cur, wave_slot, 1, mw);
        }
    };
    // (s_idx, r) = divmod(bt, blks_per_snr), advanced incrementally (no 64-bit division per tile).
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
        // Inactive lanes (ragged tail) read row 0 and zero it: unconditional loads, no branches.
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
        MfmaAcc A;
        A.init();
        // At least one chunk (M >= 32): a do-while leaves no zero-trip path, on which the
        // compiler would materialise the accumulators' zeros a second time every batch.
        int ch = 0;
        do {
            const int t0 = ch * chunk_tiles;
            const int cnt = min(chunk_tiles, ntiles - t0);
            if (nchunks > 1) {
                __syncthreads();
                stage(t0, cnt);
                __syncthreads();
            }
            mfma_tiles<T, D, SPLIT>(lds_frag, lane, t0, cnt, b.m, bfr, A);
        } while (++ch < nchunks);
        float g, mi;
        mfma_epilogue<T, D, SPLIT>(b, k, pv, bfr, A, n, active, bad, txl, lane, g, mi);
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
hipError_t launch_t(const LaunchArgs& a, const void* frag, const void* pv, int grid, hipStream_t st) {
    constexpr int S = Slots<D, SPLIT>::S;
    const int ntiles = a.M >> 5;
    const int chunk_tiles = std::min(ntiles, kMfmaLdsBytes / (S * 64 * 16));
    const size_t lds = (size_t)mfma_lds_tiles(chunk_tiles) * S * 64 * 16;
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
    if (mfma_small_supported(a.M, a.D)) return launch_demap_mfma_small(a, prec, frag, pv, grid, st);
    switch (prec) {
        case 1: return launch_d<__bf16, false>(a, frag, pv, grid, st);
        case 2: return launch_d<_Float16, false>(a, frag, pv, grid, st);
        case 3: return launch_d<__bf16, true>(a, frag, pv, grid, st);
        case 4: return launch_d<_Float16, true>(a, frag, pv, grid, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace dm
