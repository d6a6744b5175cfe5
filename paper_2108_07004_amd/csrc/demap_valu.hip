// Exact soft demapper, FP32 direct-difference variant, plus the far-subset fix-up (gfx950).
//
// One lane owns one received symbol and walks the whole label-ordered point table, which is
// staged in LDS and read with wave-uniform addresses (broadcast); the per-symbol arithmetic is
// in valu_body.hpp.  A persistent grid walks (SNR point, 512-symbol tile) work items.
#include "device_common.hpp"
#include "fixup_drain.hpp"
#include "kernels.hpp"
#include "valu_body.hpp"

namespace dm {

namespace {

constexpr int kValuThreads = 512;
constexpr int kLdsFloats = 16384;  // 64 KiB of points per staged chunk

template <int DP>
__global__ __launch_bounds__(kValuThreads) void demap_valu_kernel(const LaunchArgs a) {
    extern __shared__ float lds[];
    const int M = a.M, D = a.D;
    const int Mpad = M < 16 ? 16 : M;
    // Chunk = whole table when it fits in 64 KiB, else a multiple of 64 points.
    int chunk = (kLdsFloats / DP) & ~63;
    if (chunk >= Mpad) chunk = Mpad;
    const int nchunks = (Mpad + chunk - 1) / chunk;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave_slot = (blockIdx.x * (kValuThreads / 64) + (tid >> 6)) % kAccSlots;
    const Sinks& k = a.sinks;

    auto stage = [&](int c0, int cnt) {
        for (int i = tid; i < cnt * DP; i += kValuThreads) {
            const int j = c0 + i / DP;
            lds[i] = (j < M) ? a.table[(size_t)c0 * DP + i] : 1.0e19f;  // padding: e_j = 0
        }
    };
    if (nchunks == 1) {
        stage(0, Mpad);
        __syncthreads();
    }

    const int64_t total = a.tiles_per_snr * a.n_snr;
    double gsum = 0.0, msum = 0.0;
    int cur = -1;
    for (int64_t tile = blockIdx.x; tile < total; tile += gridDim.x) {
        const int s = (int)(tile / a.tiles_per_snr);
        const int64_t n = (tile % a.tiles_per_snr) * kValuThreads + tid;
        if (s != cur) {
            if (cur >= 0 && k.acc && lane == 0) {
                acc_add(k.acc, cur, wave_slot, 0, gsum);
                acc_add(k.acc, cur, wave_slot, 1, msum);
            }
            gsum = msum = 0.0;
            cur = s;
        }
        const bool active = n < a.N;
        const BlockView b = view_sym(a, s, n, active);
        float y[DP];
        load_symbol<DP>(y, b.y + (size_t)(active ? n : 0) * D, D, active);

        DM_VALU_ACC_DECL
        for (int ch = 0; ch < nchunks; ++ch) {
            const int c0 = ch * chunk;
            const int cnt = min(chunk, Mpad - c0);
            if (nchunks > 1) {
                __syncthreads();
                stage(c0, cnt);
                __syncthreads();
            }
            valu_accumulate<DP>(lds, c0, cnt, y, b.c, b.K, b.m, accA, accB, hi0, hi1);
        }
        float g, mi;
        valu_epilogue<DP>(b, k, n, active, y, accA, accB, hi0, hi1, g, mi);
        if (k.acc) {
            gsum += wave_sum(active ? (double)g : 0.0);
            msum += wave_sum(active ? (double)mi : 0.0);
        }
    }
    if (cur >= 0 && k.acc && lane == 0) {
        acc_add(k.acc, cur, wave_slot, 0, gsum);
        acc_add(k.acc, cur, wave_slot, 1, msum);
    }
}

// Exact recomputation of the queued symbols (one lane or one wavefront per symbol).
template <int DP>
__global__ __launch_bounds__(256) void fixup_kernel(const LaunchArgs a, int cache_pts) {
    extern __shared__ float s_t[];  // per-wave exponent caches, 4 x cache_pts floats
    drain_fix_queue<DP>(a.sinks, [&](const FixEntry& e) { return view_sym(a, (int)e.tag, e.n, true); },
                        s_t + (threadIdx.x >> 6) * cache_pts, cache_pts, a.M, a.table);
}

template <int DP>
hipError_t launch_valu_t(const LaunchArgs& a, int grid, hipStream_t st) {
    const int Mpad = a.M < 16 ? 16 : a.M;
    int chunk = (kLdsFloats / DP) & ~63;
    if (chunk >= Mpad) chunk = Mpad;
    const size_t lds = (size_t)chunk * DP * sizeof(float);
    hipLaunchKernelGGL(demap_valu_kernel<DP>, dim3(grid), dim3(kValuThreads), lds, st, a);
    return hipGetLastError();
}

template <int DP>
hipError_t launch_fixup_t(const LaunchArgs& a, int grid, hipStream_t st) {
    hipLaunchKernelGGL(fixup_kernel<DP>, dim3(grid), dim3(256), fixup_lds_bytes(a.M), st, a, fixup_cache_points(a.M));
    return hipGetLastError();
}

}  // namespace

int padded_dim(int D) {
    if (D <= 8) return D;
    return D <= 16 ? 16 : 32;
}

int valu_tile_symbols() { return kValuThreads; }

#define DM_DISPATCH_DP(FN, ...)                          \
    switch (padded_dim(a.D)) {                          \
        case 1: return FN<1>(__VA_ARGS__);              \
        case 2: return FN<2>(__VA_ARGS__);              \
        case 3: return FN<3>(__VA_ARGS__);              \
        case 4: return FN<4>(__VA_ARGS__);              \
        case 5: return FN<5>(__VA_ARGS__);              \
        case 6: return FN<6>(__VA_ARGS__);              \
        case 7: return FN<7>(__VA_ARGS__);              \
        case 8: return FN<8>(__VA_ARGS__);              \
        case 16: return FN<16>(__VA_ARGS__);            \
        case 32: return FN<32>(__VA_ARGS__);            \
        default: return hipErrorInvalidValue;           \
    }

hipError_t launch_demap_valu(const LaunchArgs& a, int grid, hipStream_t st) {
    DM_DISPATCH_DP(launch_valu_t, a, grid, st)
}

hipError_t launch_fixup(const LaunchArgs& a, int grid, hipStream_t st) {
    DM_DISPATCH_DP(launch_fixup_t, a, grid, st)
}

}  // namespace dm
