// Batched exact demapping: one persistent launch over many (constellation, noise level, block)
// instances of uneven M, D and N (gfx950).
//
// Work items are (instance, sub consecutive symbol tiles) pairs listed instance by instance,
// the most costly instance first (sub per instance, from the plan's shape choice).  Workgroups claim fixed chunks of `grab` consecutive items from a counter
// (dynamic balance: the cheap items at the end fill the tail) and restage their LDS table only
// when the next item belongs to another instance.  GMI / MI partial sums are flushed per chunk
// and instance, so every fixed-point contribution covers a fixed set of symbols whichever
// workgroup runs it: the totals are bit-reproducible.  Each instance runs either
// the FP32 direct-difference body (one lane per symbol, 1024-symbol tiles) or the MFMA body
// (one wave per 32 symbols, 512-symbol tiles; 32..256-point constellations take the
// compile-time tile loop of mfma_small.hpp), as chosen per (M, D) by the autotuner.  Batched
// tables use a row stride of 8 (D <= 8 zero-padded): the padded coordinates contribute exact
// zeros, and the MFMA operand vectors of every instance have the same K layout.
#include "device_common.hpp"
#include "fixup_drain.hpp"
#include "kernels.hpp"
#include "mfma_body.hpp"
#include "mfma_small.hpp"
#include "valu_body.hpp"

namespace dm {

namespace {

constexpr int kThreads = 1024;
constexpr int kWaves = kThreads / 64;

// One 32-symbol batch of an instance with 32 * NT points (D padded to 8): compile-time tile loop
// and epilogue.
template <typename T, bool SPLIT, int NT>
__device__ __forceinline__ void small_item(const uint4* lds, const BlockView& b, const Sinks& k, const uint16_t* pv,
                                           const Frags<T, Slots<8, SPLIT>::S>& bfr, int64_t n, bool active, bool bad,
                                           int txl, int lane, float& g, float& mi) {
    constexpr int MB = SmallBits<NT>::MB;
    float S0[MB], S1[MB], tot;
    mfma_small_sums<T, 8, SPLIT, NT>(lds, lane, bfr, S0, S1, tot);
    mfma_finish<T, 8, SPLIT, MB>(b, k, pv, bfr, S0, S1, tot, n, active, bad, txl, lane, g, mi);
}

template <typename T, bool SPLIT>
__global__ __launch_bounds__(kThreads) void demap_batched_kernel(const BatchArgs a) {
    extern __shared__ uint4 lds_raw[];
    constexpr int S = Slots<8, SPLIT>::S;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int h = lane >> 5;
    const int wave = tid >> 6;
    const int wave_slot = (blockIdx.x * kWaves + wave) % kAccSlots;  // integer slots: any spread sums alike
    const Sinks& k = a.sinks;
    __shared__ int s_claim;
    int staged = -1;
    for (;;) {
        if (tid == 0) s_claim = (int)atomicAdd(a.next, (uint32_t)a.grab);
        __syncthreads();
        const int i0 = s_claim;
        __syncthreads();  // every thread has read the claim before it is overwritten
        if (i0 >= a.n_items) break;
        const int i1 = min(i0 + a.grab, a.n_items);
        int cur = -1;
        double gsum = 0.0, msum = 0.0;
        for (int i = i0; i < i1; ++i) {
            const WorkItem it = a.items[i];
            const int inst = it.inst;
            const BatchDesc& d = a.desc[inst];
            const BlockView b = d.view;
            const int kind = d.kind;
            if (inst != staged) {  // restage the point table (whole block, uniform condition)
                __syncthreads();
                if (kind == kKindMfma) {
                    const int n16 = (b.M >> 5) * S * 64;
                    for (int j = tid; j < n16; j += kThreads) lds_raw[j] = d.frag[j];
                } else {
                    float* lds = reinterpret_cast<float*>(lds_raw);
                    const int Mpad = b.M < 16 ? 16 : b.M;
                    for (int j = tid; j < Mpad * 8; j += kThreads)
                        lds[j] = (j < b.M * 8) ? b.table[j] : 1.0e19f;  // padding rows: e_j = 0
                }
                __syncthreads();
                staged = inst;
            }
            if (inst != cur) {
                if (cur >= 0 && k.acc && lane == 0) {
                    acc_add(k.acc, cur, wave_slot, 0, gsum);
                    acc_add(k.acc, cur, wave_slot, 1, msum);
                }
                gsum = msum = 0.0;
                cur = inst;
            }
            // The item's sub symbol tiles; GMI / MI terms summed per lane, then over the wave once.
            double gl = 0.0, ml = 0.0;
            for (int sb = 0; sb < d.sub; ++sb) {
                float g = 0.0f, mi = 0.0f;
                bool active;
                if (kind == kKindMfma) {
                    const int64_t n = it.n0 + (int64_t)sb * (kWaves * 32) + wave * 32 + (lane & 31);
                    active = n < b.N;
                    float y[8];
                    load_symbol<8>(y, b.y + (size_t)(active ? n : 0) * b.D, b.D, active);
                    bool bad = false;
                    const Frags<T, S> bfr = build_symbol_frags<T, 8, SPLIT>(y, b.c, b.K, h, bad);
                    const int txl = (b.tx && active) ? tx_label(b, k, n) : 0;
                    switch (b.M) {  // uniform: 32..256 points take the compile-time tile loop
                        case 32: small_item<T, SPLIT, 1>(lds_raw, b, k, d.pv, bfr, n, active, bad, txl, lane, g, mi); break;
                        case 64: small_item<T, SPLIT, 2>(lds_raw, b, k, d.pv, bfr, n, active, bad, txl, lane, g, mi); break;
                        case 128: small_item<T, SPLIT, 4>(lds_raw, b, k, d.pv, bfr, n, active, bad, txl, lane, g, mi); break;
                        case 256: small_item<T, SPLIT, 8>(lds_raw, b, k, d.pv, bfr, n, active, bad, txl, lane, g, mi); break;
                        default: {
                            MfmaAcc A;
                            A.init();
                            mfma_tiles<T, 8, SPLIT>(lds_raw, lane, 0, b.M >> 5, b.m, bfr, A);
                            mfma_epilogue<T, 8, SPLIT>(b, k, d.pv, bfr, A, n, active, bad, txl, lane, g, mi);
                        }
                    }
                } else {
                    const int64_t n = it.n0 + (int64_t)sb * kThreads + tid;
                    active = n < b.N;
                    float y[8];
                    load_symbol<8>(y, b.y + (size_t)(active ? n : 0) * b.D, b.D, active);
                    DM_VALU_ACC_DECL
                    const int Mpad = b.M < 16 ? 16 : b.M;
                    valu_accumulate<8>(reinterpret_cast<const float*>(lds_raw), 0, Mpad, y, b.c, b.K, b.m, accA, accB,
                                       hi0, hi1);
                    valu_epilogue<8>(b, k, n, active, y, accA, accB, hi0, hi1, g, mi);
                }
                if (active) {
                    gl += (double)g;
                    ml += (double)mi;
                }
            }
            if (k.acc) {
                gsum += wave_sum(gl);
                msum += wave_sum(ml);
            }
        }
        if (cur >= 0 && k.acc && lane == 0) {
            acc_add(k.acc, cur, wave_slot, 0, gsum);
            acc_add(k.acc, cur, wave_slot, 1, msum);
        }
    }
}

// Exact recomputation of the queued symbols of every instance (one lane or one wavefront per symbol).
__global__ __launch_bounds__(256) void batched_fixup_kernel(const BatchArgs a) {
    __shared__ float s_t[4][kFixCached];  // per-wave exponent cache (32 KiB per block)
    drain_fix_queue<8>(a.sinks, [&](const FixEntry& e) { return a.desc[e.tag].view; }, s_t[threadIdx.x >> 6],
                       kFixCached);
}

// Zero the accumulators and counters with a kernel (a graph must not hold memset nodes).
__global__ void zero_words(uint32_t* p, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

template <typename T, bool SPLIT>
hipError_t prepare_t() {
    return hipFuncSetAttribute((const void*)demap_batched_kernel<T, SPLIT>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               kBatchedLdsAlloc);
}

template <typename T, bool SPLIT>
hipError_t launch_batched_t(const BatchArgs& a, int grid, hipStream_t st) {
    hipLaunchKernelGGL((demap_batched_kernel<T, SPLIT>), dim3(grid), dim3(kThreads), kBatchedLdsAlloc, st, a);
    return hipGetLastError();
}

}  // namespace

int batched_tile_symbols(int kind) { return kind == kKindMfma ? kWaves * 32 : kThreads; }

hipError_t launch_demap_batched(const BatchArgs& a, int prec, int grid, hipStream_t st) {
    switch (prec) {
        case 0:  // FP32: every instance runs the VALU body; the MFMA operand type is unused
        case 4: return launch_batched_t<_Float16, true>(a, grid, st);
        case 1: return launch_batched_t<__bf16, false>(a, grid, st);
        case 2: return launch_batched_t<_Float16, false>(a, grid, st);
        case 3: return launch_batched_t<__bf16, true>(a, grid, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t prepare_batched(int prec) {
    switch (prec) {
        case 0:
        case 4: return prepare_t<_Float16, true>();
        case 1: return prepare_t<__bf16, false>();
        case 2: return prepare_t<_Float16, false>();
        case 3: return prepare_t<__bf16, true>();
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_batched_fixup(const BatchArgs& a, int grid, hipStream_t st) {
    hipLaunchKernelGGL(batched_fixup_kernel, dim3(grid), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_zero_words(uint32_t* p, size_t n, hipStream_t st) {
    hipLaunchKernelGGL(zero_words, dim3(64), dim3(256), 0, st, p, n);
    return hipGetLastError();
}

}  // namespace dm
