// Minimum-distance decisions with the distance cross term on MFMA (gfx950), exact by proof.
//
// The split-FP16 MFMA (three products per term, FP32 accumulation) yields for every symbol and
// point u~ = K + 2 y.x - ||x||^2 - ||y||^2 = K - ||y - x||^2, with a per-symbol offset
// K = (||y|| + r_max)^2 + 1 that keeps every u~ positive, so the bit patterns of the u~ order
// like their values.  Register r of tile t holds label 32 t + 16 h + r; each lane keeps, per
// register slot r, the largest and second-largest values with the (complemented) tile index
// written into their low 7 mantissa bits.  Tiles are taken in pairs: with a, b the slot's two
// new values, best = max3(best, a, b) and second = max(second, med3(best, a, b)) (the second
// largest of {best, second, a, b}, as second <= best): with the field inserts, five vector
// instructions per two (symbol, point) pairs, all unsigned integer max / med3 / bit operations.  Per value, |u~ - u| is at most 3.5e-6 K (FP32 accumulation of
// 3D + 5 terms bounded by 2K) + 1e-6 K (operand splitting, dropped lo*lo products) + 5.4e-7 K
// (rounding of the reference FP32 distance) + 7.6e-6 K (the 7 packed bits), under 1.3e-5 K in
// all; with eps = 2^-14 K (+ a floor for FP16 subnormal lo parts) a gap best - second > 2 eps
// proves the winner is the unique minimiser of the reference FP32 distance, so it is the
// decision.  Otherwise (near or exact ties, values out of FP16 range, non-finite inputs) the
// symbol is queued and hard_fix_kernel decides it with the reference formula itself (lowest
// label among equal distances).
#include "device_common.hpp"
#include "kernels.hpp"
#include "mfma_body.hpp"

namespace dm {

namespace {

constexpr int kHardMfmaThreads = 1024;
constexpr int kHardMfmaLds = 131072;
constexpr uint32_t kTileMask = 0x7Fu;  // packed tile index: M <= 4096 (t < 128)

// Reference FP32 distance of the library's hard decisions.
template <int DP>
__device__ __forceinline__ float ref_dist(const float (&y)[DP], const float* x) {
    float acc = 0.0f;
#pragma unroll
    for (int d = 0; d < DP; ++d) {
        const float t = y[d] - x[d];
        acc = __builtin_fmaf(t, t, acc);
    }
    return acc;
}

// Exact decision of one symbol by one lane (queue overflow path).
template <int DP>
__device__ int lane_exact(const float (&y)[DP], const float* table, int M) {
    float best = __builtin_inff();
    int arg = 0;
    for (int j = 0; j < M; ++j) {
        const float d = ref_dist<DP>(y, table + (size_t)j * DP);
        if (d < best) {
            best = d;
            arg = j;
        }
    }
    return arg;
}

template <int D>
__global__ __launch_bounds__(kHardMfmaThreads) void hard_mfma_kernel(const HardArgs a, const uint4* __restrict__ frag,
                                                                     float r_max, FixEntry* queue,
                                                                     uint32_t* queue_count, uint32_t queue_cap) {
    using T = _Float16;
    constexpr int S = Slots<D, true>::S;
    using V = typename Mma<T>::V;
    extern __shared__ uint4 lds_frag[];
    const int ntiles = a.M >> 5;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int h = lane >> 5;
    const int wave = tid >> 6;
    constexpr int kWaves = kHardMfmaThreads / 64;
    const int chunk_tiles = min(ntiles, kHardMfmaLds / (S * 64 * 16));
    const int nchunks = (ntiles + chunk_tiles - 1) / chunk_tiles;
    auto stage = [&](int t0, int cnt) {
        const uint4* src = frag + (size_t)t0 * S * 64;
        for (int i = tid; i < cnt * S * 64; i += kHardMfmaThreads) lds_frag[i] = src[i];
    };
    if (nchunks == 1) {
        stage(0, ntiles);
        __syncthreads();
    }
    const int64_t sym_per_blk = (int64_t)kWaves * 32;
    const int64_t blks = (a.N + sym_per_blk - 1) / sym_per_blk;
    const int64_t total = blks * a.n_blk;
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
    for (int64_t bt = blockIdx.x; bt < total; bt += gridDim.x) {
        const int s = (int)(bt / blks);
        const int64_t n = (bt % blks) * sym_per_blk + wave * 32 + (lane & 31);
        if (s != cur) {
            flush();
            cur = s;
        }
        const bool active = n < a.N;
        float y[D];
#pragma unroll
        for (int d = 0; d < D; ++d) y[d] = active ? a.y[s][(size_t)n * D + d] : 0.0f;
        float ysq = 0.0f;
#pragma unroll
        for (int d = 0; d < D; ++d) ysq = fmaf(y[d], y[d], ysq);
        const float rr = sqrtf(ysq) + r_max;
        const float K = fmaf(rr, rr, 1.0f);
        bool bad = false;
        const Frags<T, S> bfr = build_symbol_frags<T, D, true>(y, 1.0f, K, h, bad);
        // per register slot r: largest and second-largest packed u~ (field = kTileMask - t)
        uint32_t best[16], sec[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) best[r] = sec[r] = 0u;
        // the mask lives in a register so that masking and inserting the (scalar) tile field is
        // one v_and_or_b32 (a literal mask and a scalar field would need two instructions)
        uint32_t keep = ~kTileMask;
        asm volatile("" : "+v"(keep));
        for (int ch = 0; ch < nchunks; ++ch) {
            const int t0 = ch * chunk_tiles;
            const int cnt = min(chunk_tiles, ntiles - t0);
            if (nchunks > 1) {
                __syncthreads();
                stage(t0, cnt);
                __syncthreads();
            }
            auto tile_mma = [&](int t) {
                const uint4* fp = lds_frag + (size_t)t * S * 64 + lane;
                f32x16 acc = Mma<T>::run(__builtin_bit_cast(V, fp[0]), bfr.v[0]);
#pragma unroll
                for (int q = 1; q < S; ++q) acc = Mma<T>::run(__builtin_bit_cast(V, fp[q * 64]), bfr.v[q], acc);
                return acc;
            };
            // Tiles t and t + 1 together.  Their MFMAs are not issued ahead of the previous pair's
            // ranking: two more accumulators would spill, and the other waves of the SIMD cover
            // the MFMA latency.
            for (int t = 0; t + 1 < cnt; t += 2) {
                const f32x16 xa = tile_mma(t), xb = tile_mma(t + 1);
                const uint32_t fa = kTileMask - (uint32_t)(t0 + t), fb = fa - 1u;
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const uint32_t a = (__float_as_uint(xa[r]) & keep) | fa;
                    const uint32_t b = (__float_as_uint(xb[r]) & keep) | fb;
                    uint32_t med;  // median of three (the compiler's own pattern match misses it here)
                    asm("v_med3_u32 %0, %1, %2, %3" : "=v"(med) : "v"(best[r]), "v"(a), "v"(b));
                    sec[r] = max(sec[r], med);
                    best[r] = max(max(best[r], a), b);
                }
            }
            if (cnt & 1) {  // the last tile of an odd count alone
                const f32x16 xa = tile_mma(cnt - 1);
                const uint32_t fa = kTileMask - (uint32_t)(t0 + cnt - 1);
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const uint32_t a = (__float_as_uint(xa[r]) & keep) | fa;
                    sec[r] = max(sec[r], min(best[r], a));
                    best[r] = max(best[r], a);
                }
            }
        }
        // this half's winner (slot r1) and runner-up, then the two halves of the symbol
        uint32_t b1 = best[0], b2 = sec[0];
        int r1 = 0;
#pragma unroll
        for (int r = 1; r < 16; ++r) {
            b2 = max(max(b2, sec[r]), min(b1, best[r]));
            r1 = best[r] > b1 ? r : r1;
            b1 = max(b1, best[r]);
        }
        const uint32_t s1 = b2;
        const uint32_t pb = __shfl_xor(b1, 32, 64), ps = __shfl_xor(s1, 32, 64);
        const int pr = __shfl_xor(r1, 32, 64);
        const bool pbad = __shfl_xor((int)bad, 32, 64);
        const uint32_t bg = max(b1, pb);
        const uint32_t sg = max(max(s1, ps), min(b1, pb));
        const bool mine = b1 >= pb;
        const int tw = (int)(kTileMask - (bg & kTileMask));
        const int label = 32 * tw + 16 * (mine ? h : 1 - h) + (mine ? r1 : pr);
        const float gap = __uint_as_float(bg & ~kTileMask) - __uint_as_float(sg & ~kTileMask);
        const float eps = 0x1p-14f * K + 0x1p-18f * (1.0f + rr);
        const bool ok = !bad && !pbad && (gap > 2.0f * eps) && (gap < __builtin_inff()) && label < a.M;
        if (h == 0 && active) {
            int dec = label;
            bool decided = ok;
            if (!ok) {
                const uint32_t slot = atomicAdd(queue_count, 1u);
                if (slot < queue_cap) {
                    queue[slot] = FixEntry{(uint32_t)n, (uint32_t)s, 0u, 0u};
                } else {
                    float yp[D];
#pragma unroll
                    for (int d = 0; d < D; ++d) yp[d] = y[d];
                    dec = lane_exact<D>(yp, a.table, a.M);
                    decided = true;
                }
            }
            if (decided) {
                if (a.labels_out[s]) a.labels_out[s][n] = (uint16_t)dec;
                if (a.counts) {
                    uint32_t row = a.tx[n];
                    if (row >= (uint32_t)a.M) {
                        atomicOr(a.bad_tx, 1u);
                        row = 0;
                    }
                    const uint32_t txl = a.row2label[row];
                    se += (uint32_t)dec != txl;
                    be += __builtin_popcount((uint32_t)dec ^ txl);
                }
            }
        }
    }
    flush();
}

// One lane per queued symbol: the reference FP32 distance to every point of the label-ordered
// table, staged in LDS and read with wave-uniform addresses (broadcast), strict "<" in label
// order (ties to the lowest label).  All threads of a block run the same number of rounds so
// the chunked staging can synchronise the block.
constexpr int kFixThreads = 256;
constexpr int kFixLdsFloats = 16384;  // 64 KiB of points per staged chunk

template <int DP>
__global__ __launch_bounds__(kFixThreads) void hard_fix_kernel(const HardArgs a, const FixEntry* queue,
                                                                const uint32_t* count_p, uint32_t cap) {
    extern __shared__ float lds[];
    __shared__ unsigned long long s_cnt[2 * kMaxSnrPerLaunch];  // per block: symbol, bit errors
    const uint32_t count = min(*count_p, cap);
    const int tid = threadIdx.x;
    for (int q = tid; q < 2 * kMaxSnrPerLaunch; q += kFixThreads) s_cnt[q] = 0ull;
    int chunk = (kFixLdsFloats / DP) & ~63;
    if (chunk >= a.M) chunk = a.M;
    const int nchunks = (a.M + chunk - 1) / chunk;
    if (nchunks == 1)
        for (int i = tid; i < a.M * DP; i += kFixThreads) lds[i] = a.table[i];
    __syncthreads();
    const uint32_t stride = gridDim.x * kFixThreads;
    const uint32_t rounds = (count + stride - 1) / stride;
    for (uint32_t rd = 0; rd < rounds; ++rd) {
        const uint32_t i = rd * stride + blockIdx.x * kFixThreads + tid;
        const bool live = i < count;
        FixEntry e{0u, 0u, 0u, 0u};
        if (live) e = queue[i];
        const int s = (int)e.tag;
        float y[DP];
        load_symbol<DP>(y, a.y[s] + (size_t)e.n * a.D, a.D, live);
        float best = __builtin_inff();
        int arg = 0;
        for (int ch = 0; ch < nchunks; ++ch) {
            const int c0 = ch * chunk;
            const int cnt = min(chunk, a.M - c0);
            if (nchunks > 1) {
                __syncthreads();
                for (int q = tid; q < cnt * DP; q += kFixThreads) lds[q] = a.table[(size_t)c0 * DP + q];
                __syncthreads();
            }
#pragma unroll 8
            for (int j = 0; j < cnt; ++j) {
                const float d = ref_dist<DP>(y, lds + j * DP);
                const bool better = d < best;
                best = better ? d : best;
                arg = better ? c0 + j : arg;
            }
        }
        if (live) {
            if (a.labels_out[s]) a.labels_out[s][e.n] = (uint16_t)arg;
            if (a.counts) {
                uint32_t row = a.tx[e.n];
                if (row >= (uint32_t)a.M) {
                    atomicOr(a.bad_tx, 1u);
                    row = 0;
                }
                const uint32_t txl = a.row2label[row];
                if ((uint32_t)arg != txl) atomicAdd(&s_cnt[2 * s], 1ull);
                const uint32_t nb = __builtin_popcount((uint32_t)arg ^ txl);
                if (nb) atomicAdd(&s_cnt[2 * s + 1], (unsigned long long)nb);
            }
        }
    }
    if (a.counts) {  // one global update per block and counter
        __syncthreads();
        for (int q = tid; q < 2 * a.n_blk; q += kFixThreads)
            if (s_cnt[q]) atomicAdd(a.counts + q, s_cnt[q]);
    }
}

template <int D>
hipError_t launch_hard_mfma_t(const HardArgs& a, const void* frag, float r_max, FixEntry* queue, uint32_t* qcount,
                              uint32_t qcap, int grid, hipStream_t st) {
    constexpr int S = Slots<D, true>::S;
    const int ntiles = a.M >> 5;
    const int chunk_tiles = std::min(ntiles, kHardMfmaLds / (S * 64 * 16));
    const size_t lds = (size_t)chunk_tiles * S * 64 * 16;
    auto kern = hard_mfma_kernel<D>;
    hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(grid), dim3(kHardMfmaThreads), lds, st, a, (const uint4*)frag, r_max, queue, qcount,
                       qcap);
    return hipGetLastError();
}

template <int DP>
hipError_t launch_hard_fix_t(const HardArgs& a, const FixEntry* queue, const uint32_t* qcount, uint32_t qcap, int grid,
                             hipStream_t st) {
    const size_t lds = sizeof(float) * (size_t)std::min(a.M * DP, kFixLdsFloats);
    hipError_t e = hipFuncSetAttribute((const void*)hard_fix_kernel<DP>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(hard_fix_kernel<DP>, dim3(grid), dim3(kFixThreads), lds, st, a, queue, qcount, qcap);
    return hipGetLastError();
}

}  // namespace

int hard_mfma_block_symbols() { return (kHardMfmaThreads / 64) * 32; }

hipError_t launch_hard_mfma(const HardArgs& a, const void* frag, float r_max, FixEntry* queue, uint32_t* qcount,
                            uint32_t qcap, int grid, hipStream_t st) {
    switch (a.D) {
        case 1: return launch_hard_mfma_t<1>(a, frag, r_max, queue, qcount, qcap, grid, st);
        case 2: return launch_hard_mfma_t<2>(a, frag, r_max, queue, qcount, qcap, grid, st);
        case 3: return launch_hard_mfma_t<3>(a, frag, r_max, queue, qcount, qcap, grid, st);
        case 4: return launch_hard_mfma_t<4>(a, frag, r_max, queue, qcount, qcap, grid, st);
        case 5: return launch_hard_mfma_t<5>(a, frag, r_max, queue, qcount, qcap, grid, st);
        case 6: return launch_hard_mfma_t<6>(a, frag, r_max, queue, qcount, qcap, grid, st);
        case 7: return launch_hard_mfma_t<7>(a, frag, r_max, queue, qcount, qcap, grid, st);
        case 8: return launch_hard_mfma_t<8>(a, frag, r_max, queue, qcount, qcap, grid, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_hard_fix(const HardArgs& a, const FixEntry* queue, const uint32_t* qcount, uint32_t qcap, int grid,
                           hipStream_t st) {
    switch (a.D) {
        case 1: return launch_hard_fix_t<1>(a, queue, qcount, qcap, grid, st);
        case 2: return launch_hard_fix_t<2>(a, queue, qcount, qcap, grid, st);
        case 3: return launch_hard_fix_t<3>(a, queue, qcount, qcap, grid, st);
        case 4: return launch_hard_fix_t<4>(a, queue, qcount, qcap, grid, st);
        case 5: return launch_hard_fix_t<5>(a, queue, qcount, qcap, grid, st);
        case 6: return launch_hard_fix_t<6>(a, queue, qcount, qcap, grid, st);
        case 7: return launch_hard_fix_t<7>(a, queue, qcount, qcap, grid, st);
        case 8: return launch_hard_fix_t<8>(a, queue, qcount, qcap, grid, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace dm
