// Hard-decision (minimum Euclidean distance) demapping with symbol- and bit-error counting
// (gfx950).  The paper's receiver decides each symbol by the minimum-distance criterion over
// the uploaded point table (Sec. 2) and reports BER-based Q-factors (Sec. 4).
//
// One lane owns one received symbol and scans the label-ordered FP32 table staged in LDS
// (wave-uniform broadcast reads).  The squared distance is accumulated as
//     t_d = y_d - x_d,  acc = fma(t_d, t_d, acc),  d = 0 .. D-1,  acc starting at 0,
// exactly in that order, so any FP32 implementation of the same formula reaches the same
// distances bit for bit and therefore the same decisions; a strict "<" over the label order
// resolves ties to the lowest label.  Errors are counted in integers (deterministic).
#include "device_common.hpp"
#include "kernels.hpp"

namespace dm {

namespace {

constexpr int kHardThreads = 512;
constexpr int kHardLdsFloats = 16384;  // 64 KiB of points per staged chunk

template <int DP>
__global__ __launch_bounds__(kHardThreads) void hard_demap_kernel(const HardArgs a) {
    extern __shared__ float lds[];
    const int M = a.M, D = a.D;
    int chunk = (kHardLdsFloats / DP) & ~63;
    if (chunk >= M) chunk = M;
    const int nchunks = (M + chunk - 1) / chunk;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    if (nchunks == 1) {
        for (int i = tid; i < M * DP; i += kHardThreads) lds[i] = a.table[i];
        __syncthreads();
    }
    const int64_t total = a.tiles_per_blk * a.n_blk;
    // Error counts accumulate per lane and go out once per received block and wave: one counter
    // address per block, and device-scope atomics on one address serialise (~11 ns each).
    uint32_t se = 0, be = 0;
    int cur = -1;
    auto flush = [&]() {
        if (cur < 0 || !a.counts) return;
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            se += __shfl_xor(se, off, 64);
            be += __shfl_xor(be, off, 64);
        }
        if (lane == 0) {
            if (se) atomicAdd(a.counts + 2 * cur, (unsigned long long)se);
            if (be) atomicAdd(a.counts + 2 * cur + 1, (unsigned long long)be);
        }
        se = be = 0;
    };
    for (int64_t tile = blockIdx.x; tile < total; tile += gridDim.x) {
        const int s = (int)(tile / a.tiles_per_blk);
        if (s != cur) {  // block-uniform
            flush();
            cur = s;
        }
        const int64_t n = (tile % a.tiles_per_blk) * kHardThreads + tid;
        const bool active = n < a.N;
        float y[DP];
        load_symbol<DP>(y, a.y[s] + (size_t)(active ? n : 0) * D, D, active);
        float best = __builtin_inff();
        int arg = 0;
        for (int ch = 0; ch < nchunks; ++ch) {
            const int c0 = ch * chunk;
            const int cnt = min(chunk, M - c0);
            if (nchunks > 1) {
                __syncthreads();
                for (int i = tid; i < cnt * DP; i += kHardThreads) lds[i] = a.table[(size_t)c0 * DP + i];
                __syncthreads();
            }
#pragma unroll 4
            for (int j = 0; j < cnt; ++j) {
                const float* x = lds + j * DP;
                float acc = 0.0f;
#pragma unroll
                for (int d = 0; d < DP; ++d) {
                    const float t = y[d] - x[d];
                    acc = __builtin_fmaf(t, t, acc);
                }
                const bool better = acc < best;
                best = better ? acc : best;
                arg = better ? c0 + j : arg;
            }
        }
        if (active && a.labels_out[s]) a.labels_out[s][n] = (uint16_t)arg;
        if (a.counts && active) {
            uint32_t row = a.tx[n];
            if (row >= (uint32_t)M) {
                atomicOr(a.bad_tx, 1u);
                row = 0;
            }
            const uint32_t txl = a.row2label[row];
            se += (uint32_t)arg != txl;
            be += __builtin_popcount((uint32_t)arg ^ txl);
        }
    }
    flush();
}

template <int DP>
hipError_t launch_hard_t(const HardArgs& a, int grid, hipStream_t st) {
    const int chunk_floats = std::min(a.M * DP, kHardLdsFloats);
    const size_t lds = (size_t)chunk_floats * sizeof(float);
    hipLaunchKernelGGL(hard_demap_kernel<DP>, dim3(grid), dim3(kHardThreads), lds, st, a);
    return hipGetLastError();
}

}  // namespace

int hard_tile_symbols() { return kHardThreads; }

hipError_t launch_hard_demap(const HardArgs& a, int grid, hipStream_t st) {
    switch (padded_dim(a.D)) {
        case 1: return launch_hard_t<1>(a, grid, st);
        case 2: return launch_hard_t<2>(a, grid, st);
        case 3: return launch_hard_t<3>(a, grid, st);
        case 4: return launch_hard_t<4>(a, grid, st);
        case 5: return launch_hard_t<5>(a, grid, st);
        case 6: return launch_hard_t<6>(a, grid, st);
        case 7: return launch_hard_t<7>(a, grid, st);
        case 8: return launch_hard_t<8>(a, grid, st);
        case 16: return launch_hard_t<16>(a, grid, st);
        case 32: return launch_hard_t<32>(a, grid, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace dm
