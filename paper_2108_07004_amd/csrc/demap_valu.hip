// Exact soft demapper, FP32 direct-difference variant, plus the far-subset fix-up (gfx950).
//
// One lane owns one received symbol and walks the whole label-ordered point table,
// which is staged in LDS and read with wave-uniform addresses (broadcast).  For every
// point j the lane forms e_j = 2^(K - c ||y - x_j||^2), c = log2(e)/(2 sigma2): the
// likelihood exp(-||y-x||^2/(2 sigma2)) rescaled by the fixed factor 2^K, so no running
// maximum is needed (e_j <= 2^K because ||y-x||^2 >= 0, and K = 123 - m keeps the sum
// of M terms below 2^123).  The per-bit subset sums S_p^0, S_p^1 come from accumulators
// indexed by the label's low bits (table in label order):
//   bits 0-3: accA[j & 15] (one add per point); group sum T over 16 points (one add);
//   bits 4-5: accB[(j >> 4) & 3] (one add per 16 points);
//   bits >= 6: the 64-point block sum added to the side given by (j >> 6).
// A subset sum under 2^(m-102) may have lost terms below FP32's normal range; such
// (symbol, bit) pairs are queued for an exact max-shifted recomputation (fix-up).
#include "device_common.hpp"
#include "kernels.hpp"

namespace dm {

namespace {

constexpr int kValuThreads = 512;
constexpr int kLdsFloats = 16384;  // 64 KiB of points per staged chunk

template <int DP>
__global__ __launch_bounds__(kValuThreads) void demap_valu_kernel(const LaunchArgs a) {
    extern __shared__ float lds[];
    const int M = a.M, m = a.m, D = a.D;
    const int Mpad = M < 16 ? 16 : M;
    // Chunk = whole table when it fits in 64 KiB, else a multiple of 64 points.
    int chunk = (kLdsFloats / DP) & ~63;
    if (chunk >= Mpad) chunk = Mpad;
    const int nchunks = (Mpad + chunk - 1) / chunk;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave_slot = (blockIdx.x * (kValuThreads / 64) + (tid >> 6)) % kAccSlots;

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
            if (cur >= 0 && a.acc && lane == 0) {
                acc_add(a.acc, cur, wave_slot, 0, gsum);
                acc_add(a.acc, cur, wave_slot, 1, msum);
            }
            gsum = msum = 0.0;
            cur = s;
        }
        const SnrArg sa = a.snr[s];
        const bool active = n < a.N;
        float y[DP];
        load_symbol<DP>(y, sa.y + (size_t)(active ? n : 0) * D, D, active);
        const float c = sa.c, K = a.K;

        float accA[16], accB[4], hi0[10], hi1[10];
#pragma unroll
        for (int i = 0; i < 16; ++i) accA[i] = 0.0f;
#pragma unroll
        for (int i = 0; i < 4; ++i) accB[i] = 0.0f;
#pragma unroll
        for (int i = 0; i < 10; ++i) hi0[i] = hi1[i] = 0.0f;

        for (int ch = 0; ch < nchunks; ++ch) {
            const int c0 = ch * chunk;
            const int cnt = min(chunk, Mpad - c0);
            if (nchunks > 1) {
                __syncthreads();
                stage(c0, cnt);
                __syncthreads();
            }
            for (int b0 = 0; b0 < cnt; b0 += 64) {
                float bt = 0.0f;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    if (b0 + q * 16 < cnt) {
                        const float* xg = lds + (size_t)(b0 + q * 16) * DP;
                        float T = 0.0f;
#pragma unroll
                        for (int r = 0; r < 16; ++r) {
                            const float e = hw_exp2(fmaf(-c, sqdist<DP>(y, xg + r * DP), K));
                            accA[r] += e;
                            T += e;
                        }
                        accB[q] += T;
                        bt += T;
                    }
                }
                const int blk = (c0 + b0) >> 6;
#pragma unroll
                for (int p = 6; p < 16; ++p) {
                    if (p < m) {
                        const bool one = (blk >> (p - 6)) & 1;
                        hi1[p - 6] += one ? bt : 0.0f;
                        hi0[p - 6] += one ? 0.0f : bt;
                    }
                }
            }
        }

        // Per-bit subset sums, LLRs, GMI / MI terms.
        const int txl = (a.tx && active) ? tx_label(a, n) : 0;
        float stot = 0.0f;
#pragma unroll
        for (int r = 0; r < 16; ++r) stot += accA[r];
        float g = 0.0f;
        uint32_t mask = 0;
        float* out = (sa.llr && active) ? sa.llr + (size_t)n * m : nullptr;
#pragma unroll
        for (int p = 0; p < 16; ++p) {
            if (p >= m) break;
            float s0 = 0.0f, s1 = 0.0f;
            if (p < 4) {
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    if ((r >> p) & 1) s1 += accA[r];
                    else s0 += accA[r];
                }
            } else if (p < 6) {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    if ((q >> (p - 4)) & 1) s1 += accB[q];
                    else s0 += accB[q];
                }
            } else {
                s0 = hi0[p - 6];
                s1 = hi1[p - 6];
            }
            const bool flagged = !(fminf(s0, s1) >= a.flag_thresh);
            const float L = log2_ratio(s1, s0);
            const int b = (txl >> p) & 1;
            if (!flagged) {
                if (out) out[m - 1 - p] = L * 0.69314718055994531f;
                g += gmi_bit_term(L, b);
            } else if (!a.want_llr && fmaxf(s0, s1) >= a.near_thresh && (b ? s1 > s0 : s0 > s1)) {
                g += 1.0f;  // |L| >= 60 with the transmitted bit on the near side: term is 1 in FP64
            } else {
                mask |= 1u << p;
            }
        }
        float mi = 0.0f;
        if (a.tx) {
            if (stot >= a.flag_thresh) {
                const float ttx = fmaf(-c, sqdist<DP>(y, a.table + (size_t)txl * DP), K);
                const int e = __builtin_amdgcn_frexp_expf(stot);
                const float mant = __builtin_amdgcn_frexp_mantf(stot);
                // m - log2(stot) + t_tx, with log2(stot) = e + log2(mant) split off exactly
                mi = ((float)(m - e) + ttx) - hw_log2(mant);
            } else {
                mask |= kMiFlag;
            }
        }
        if (mask && active) {
            if (a.fix_pairs) atomicAdd(a.fix_pairs + s, (uint32_t)__popc(mask & 0xFFFFu));
            const uint32_t slot = atomicAdd(a.queue_count, 1u);
            if (slot < a.queue_cap) {
                a.queue[slot] = FixEntry{(uint32_t)n, (uint32_t)s, mask, 0u};
            } else {  // queue full: recompute in place (slow, still exact)
                double gc = 0.0, mc = 0.0;
                fixup_one<DP>(a, FixEntry{(uint32_t)n, (uint32_t)s, mask, 0u}, gc, mc);
                g += (float)gc;
                mi += (float)mc;
            }
        }
        if (a.acc) {
            const double gw = wave_sum(active ? (double)g : 0.0);
            const double mw = wave_sum(active ? (double)mi : 0.0);
            gsum += gw;
            msum += mw;
        }
    }
    if (cur >= 0 && a.acc && lane == 0) {
        acc_add(a.acc, cur, wave_slot, 0, gsum);
        acc_add(a.acc, cur, wave_slot, 1, msum);
    }
}

template <int DP>
__global__ __launch_bounds__(256) void fixup_kernel(const LaunchArgs a) {
    const uint32_t count = min(*a.queue_count, a.queue_cap);
    const uint32_t stride = gridDim.x * blockDim.x;
    const int slot = (blockIdx.x * 4 + (threadIdx.x >> 6)) % kAccSlots;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) {
        const FixEntry e = a.queue[i];
        double gc = 0.0, mc = 0.0;
        fixup_one<DP>(a, e, gc, mc);
        if (a.acc) {
            acc_add(a.acc, (int)e.snr, slot, 0, gc);
            acc_add(a.acc, (int)e.snr, slot, 1, mc);
        }
    }
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
    hipLaunchKernelGGL(fixup_kernel<DP>, dim3(grid), dim3(256), 0, st, a);
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
