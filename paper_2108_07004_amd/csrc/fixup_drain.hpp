// Draining the fix-up queue (gfx950): the exact recomputation of queued symbols by the fix-up
// kernels, one lane, one 16-lane row or one wavefront per symbol.  The queue itself, its entries
// and the in-place path of a full region are in device_common.hpp, which every demapping kernel
// includes; this file only the fix-up kernels do.
#pragma once
#include "device_common.hpp"

namespace dm {

// ---- wave-cooperative fix-up: one wavefront per queued symbol, lanes split the points ----

// Wave-wide max / sum of one float per lane, every lane receiving the result, in VALU only
// (the whole wave must be active): v_permlane32_swap and v_permlane16_swap pair lanes 32 and 16
// apart (the two outputs hold the pair in both lanes), then DPP row rotations by 8, 4, 2, 1
// combine the 16 lanes of each row.  No LDS round trips on the fix-up's dependent chains.
template <int CTRL>
__device__ __forceinline__ float dpp_f(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
}

template <typename Op>
__device__ __forceinline__ float wave_reduce_f(float v, Op op) {
    const uint32_t u = __builtin_bit_cast(uint32_t, v);
    const auto a = __builtin_amdgcn_permlane32_swap(u, u, false, false);
    v = op(__builtin_bit_cast(float, (uint32_t)a[0]), __builtin_bit_cast(float, (uint32_t)a[1]));
    const uint32_t w = __builtin_bit_cast(uint32_t, v);
    const auto b = __builtin_amdgcn_permlane16_swap(w, w, false, false);
    v = op(__builtin_bit_cast(float, (uint32_t)b[0]), __builtin_bit_cast(float, (uint32_t)b[1]));
    v = op(v, dpp_f<0x128>(v));  // row_ror:8
    v = op(v, dpp_f<0x124>(v));  // row_ror:4
    v = op(v, dpp_f<0x122>(v));  // row_ror:2
    v = op(v, dpp_f<0x121>(v));  // row_ror:1
    return v;
}

__device__ __forceinline__ float wave_max_f(float v) {
    return wave_reduce_f(v, [](float x, float y) { return fmaxf(x, y); });
}

__device__ __forceinline__ float wave_sum_f(float v) {
    return wave_reduce_f(v, [](float x, float y) { return x + y; });
}

// Exact subset log-sum-exps of label bit p (p < 0: all points into subset 0) for one symbol,
// computed by the whole wavefront; returns (log2 S^1 - log2 S^0) and, via lse0, log2 S^0.
template <int DP>
__device__ float wave_exact_llr2(const float (&y)[DP], const float* table, int M, int p, float c, float K,
                                 float& lse0) {
    const int lane = threadIdx.x & 63;
    float mx0 = -INFINITY, mx1 = -INFINITY;
    for (int j = lane; j < M; j += 64) {
        const float t = fmaf(-c, sqdist<DP>(y, table + (size_t)j * DP), K);
        if (p >= 0 && ((j >> p) & 1)) mx1 = fmaxf(mx1, t);
        else mx0 = fmaxf(mx0, t);
    }
    mx0 = wave_max_f(mx0);
    mx1 = wave_max_f(mx1);
    float s0 = 0.0f, s1 = 0.0f;
    for (int j = lane; j < M; j += 64) {
        const float t = fmaf(-c, sqdist<DP>(y, table + (size_t)j * DP), K);
        if (p >= 0 && ((j >> p) & 1)) s1 += hw_exp2(t - mx1);
        else s0 += hw_exp2(t - mx0);
    }
    s0 = wave_sum_f(s0);
    s1 = wave_sum_f(s1);
    lse0 = mx0 + hw_log2(s0);
    return (mx1 - mx0) + (hw_log2(s1) - hw_log2(s0));
}

// Exponents t_j = K - c ||y - x_j||^2 of the queued symbol, cached in the wave's LDS slice
// when M <= kFixCached (each lane keeps its own points j = lane + 64 i), so that each flagged
// bit costs one max pass and one exp2 pass over the cache instead of two passes of distance
// arithmetic.  The per-lane order of points and the wave reductions are those of
// wave_exact_llr2: same results.

__device__ __forceinline__ float cached_exact_llr2(const float* tl, int M, int p, float& lse0) {
    const int lane = threadIdx.x & 63;
    float mx0 = -INFINITY, mx1 = -INFINITY;
    for (int j = lane; j < M; j += 64) {
        const float t = tl[j];
        if (p >= 0 && ((j >> p) & 1)) mx1 = fmaxf(mx1, t);
        else mx0 = fmaxf(mx0, t);
    }
    mx0 = wave_max_f(mx0);
    mx1 = wave_max_f(mx1);
    float s0 = 0.0f, s1 = 0.0f;
    for (int j = lane; j < M; j += 64) {
        const float t = tl[j];
        if (p >= 0 && ((j >> p) & 1)) s1 += hw_exp2(t - mx1);
        else s0 += hw_exp2(t - mx0);
    }
    s0 = wave_sum_f(s0);
    s1 = wave_sum_f(s1);
    lse0 = mx0 + hw_log2(s0);
    return (mx1 - mx0) + (hw_log2(s1) - hw_log2(s0));
}

// Recompute the flagged bits (and the MI term if asked) of one queued symbol with a whole
// wavefront; lane 0 receives the GMI-term and MI-term corrections.  tl: this wave's LDS slice
// of cache_pts (<= kFixCached) floats.
template <int DP>
__device__ void fixup_wave(const BlockView& b, const Sinks& k, uint32_t n, uint32_t mask, float* tl, int cache_pts,
                           double& gcorr, double& mcorr) {
    const int lane = threadIdx.x & 63;
    float y[DP];
    load_symbol<DP>(y, b.y + (size_t)n * b.D, b.D, true);
    const int txl = b.tx ? tx_label(b, k, n) : 0;
    const bool cached = b.M <= cache_pts;  // uniform
    if (cached)
        for (int j = lane; j < b.M; j += 64) tl[j] = fmaf(-b.c, sqdist<DP>(y, b.table + (size_t)j * DP), b.K);
    for (int p = 0; p < b.m; ++p) {
        if (!((mask >> p) & 1u)) continue;
        float lse0;
        const float L = cached ? cached_exact_llr2(tl, b.M, p, lse0)
                               : wave_exact_llr2<DP>(y, b.table, b.M, p, b.c, b.K, lse0);
        if (lane == 0) {
            if (b.llr) b.llr[(size_t)n * b.m + (b.m - 1 - p)] = L * 0.69314718055994531f;
            if (b.tx) gcorr += (double)gmi_bit_term(L, (txl >> p) & 1);
        }
    }
    if ((mask & kMiFlag) && b.tx) {
        float lse_all;
        if (cached) (void)cached_exact_llr2(tl, b.M, -1, lse_all);
        else (void)wave_exact_llr2<DP>(y, b.table, b.M, -1, b.c, b.K, lse_all);
        const float ttx = fmaf(-b.c, sqdist<DP>(y, b.table + (size_t)txl * DP), b.K);
        if (lane == 0) mcorr += (double)((float)b.m - (lse_all - ttx));
    }
}

// Sum / max over the 16 lanes of each row (DPP row rotations by 8, 4, 2, 1): every lane of the
// row receives its row's result.  The whole wave must be active.
template <typename Op>
__device__ __forceinline__ float row_reduce_f(float v, Op op) {
    v = op(v, dpp_f<0x128>(v));  // row_ror:8
    v = op(v, dpp_f<0x124>(v));  // row_ror:4
    v = op(v, dpp_f<0x122>(v));  // row_ror:2
    v = op(v, dpp_f<0x121>(v));  // row_ror:1
    return v;
}

// Row fix-up for a constellation of M = 16 * NPL points (M = 128 or 256, the same for every
// queued symbol): each 16-lane row of a wavefront takes one queued symbol, so a wavefront
// recomputes four at once.  Lane r of a row keeps the exponents t = K - c ||y - x_j||^2 of labels
// j = r + 16 q in registers (less the flag bound m - 102); label bits 0-3 of j are bits of r,
// bits 4 and up bits of q.  The bit loop is unrolled, so every subset split is known at compile
// time: for p < 4 a lane's 16 values all lie in one subset, for p >= 4 the registers split in
// halves.  When the queue entry carries the near-subset log-sum (FixEntry.near) and the far side
// of the bit (mask bit kFarShift + p), only the far subset is summed, under the flag bound its
// terms all lie below (no maxima), and L = (far log-sum) - (near log-sum) with the sign of the
// far bit; otherwise both subsets are summed under their own maxima (the two-pass log-sum-exp
// of wave_exact_llr2).  Lane 0 of the row writes the LLR and accumulates the GMI / MI
// corrections, which add(tag, slot, which, value) receives.
//
// A wave's four rows run the bit loop for the union of their flagged bits, so the queue is taken
// in chunks of 512 entries per workgroup (256 threads, two entries each), each chunk
// counting-sorted by the low eight mask bits in LDS before its rows are dealt out: rows of a wave
// then mostly share their flagged bits.  The processing order does not change any result (each (symbol, bit) is written
// once, the corrections are integer sums).
constexpr int kFixSortChunk = 256;  // threads per workgroup and sort bins (low eight mask bits)
constexpr int kFixRowChunk = 512;   // entries per chunk: two per thread, so more rows share a mask

template <int DP, int NPL, typename ViewFn, typename AddFn, typename FetchFn, typename CountFn>
__device__ void fix_rows(const Sinks& k, ViewFn view, AddFn add, FetchFn fetch, CountFn count_pairs, uint32_t count,
                         const float* table) {
    constexpr int m = NPL == 8 ? 7 : 8;
    static_assert(NPL == 8 || NPL == 16, "row fix-up covers M = 128 and 256");
    // The point table (every queued symbol's, label order) in LDS: each row reads all of it, and
    // from global memory those NPL loads per lane and symbol were the kernel's latency bound.
    constexpr int kTab = DP <= 8 ? 16 * NPL * DP : 1;
    __shared__ __align__(16) float s_tab[kTab];
    const float* tab = table;
    if constexpr (DP <= 8) {
        for (int i = threadIdx.x; i < kTab; i += blockDim.x) s_tab[i] = table[i];
        __syncthreads();
        tab = s_tab;
    }
    __shared__ FixEntry s_sorted[kFixRowChunk];
    __shared__ uint32_t s_bin[256];
    __shared__ uint32_t s_wsum[kFixSortChunk / 64];
    const int tid = threadIdx.x;  // blockDim.x == kFixSortChunk
    const int lane = tid & 63;
    const int r = lane & 15;
    const int wv = tid >> 6;
    const uint32_t wave = blockIdx.x * (blockDim.x >> 6) + wv;
    const int slot = (int)(wave % kAccSlots);
    const auto fmax2 = [](float a, float b) { return fmaxf(a, b); };
    const auto fadd2 = [](float a, float b) { return a + b; };
    constexpr int kPer = kFixRowChunk / kFixSortChunk;
    for (uint32_t c0 = blockIdx.x * kFixRowChunk; c0 < count; c0 += gridDim.x * kFixRowChunk) {  // uniform per block
        const uint32_t nc = min((uint32_t)kFixRowChunk, count - c0);
        // counting sort of the chunk by key = low 8 mask bits
        s_bin[tid] = 0u;
        __syncthreads();
        FixEntry mine[kPer];
        uint32_t key[kPer];
        bool have[kPer];  // an entry with bits left to recompute
#pragma unroll
        for (int q = 0; q < kPer; ++q) {
            const uint32_t idx = (uint32_t)(tid + q * kFixSortChunk);
            mine[q] = FixEntry{};
            key[q] = 0u;
            have[q] = false;
            if (idx < nc) {
                mine[q] = fetch(c0 + idx);
                count_pairs(mine[q]);
                have[q] = (mine[q].mask & (0xFFFFu | kMiFlag)) != 0u;
            }
            if (have[q]) {
                key[q] = mine[q].mask & 0xFFu;
                atomicAdd(&s_bin[key[q]], 1u);
            }
        }
        __syncthreads();
        const uint32_t own = s_bin[tid];
        uint32_t x = own;  // inclusive scan over the 256 bins: waves, then across waves
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t y = __shfl_up(x, off, 64);
            if (lane >= off) x += y;
        }
        if (lane == 63) s_wsum[wv] = x;
        __syncthreads();
        uint32_t pre = 0u, nl = 0u;  // nl: entries dealt out as rows
        for (int w = 0; w < kFixSortChunk / 64; ++w) {
            if (w < wv) pre += s_wsum[w];
            nl += s_wsum[w];
        }
        s_bin[tid] = x + pre - own;  // exclusive start of bin tid
        __syncthreads();
#pragma unroll
        for (int q = 0; q < kPer; ++q)
            if (have[q]) s_sorted[atomicAdd(&s_bin[key[q]], 1u)] = mine[q];
        __syncthreads();
        for (uint32_t base = (uint32_t)wv * 4; base < nl; base += (blockDim.x >> 6) * 4) {  // uniform over the wave
            const uint32_t i = base + (uint32_t)(lane >> 4);
            const bool live = i < nl;
            const FixEntry e = s_sorted[live ? i : base];  // a spare row repeats a valid entry, masked off
            const uint32_t mask = live ? e.mask : 0u;
            const float near_lse = __builtin_bit_cast(float, e.near);
            const bool has_near = e.near != kNearNone;
            const BlockView b = view(e);
            float y[DP];
            load_symbol<DP>(y, b.y + (size_t)e.n * b.D, b.D, true);
            const int txl = b.tx ? tx_label(b, k, e.n) : 0;
            // Exponents relative to the flag bound sh = m - 102, below which every term of a far
            // subset lies: u_j = t_j - sh = (K - sh) - c ||y - x_j||^2.
            constexpr float sh = (float)(m - 102);
            float u[NPL];
#pragma unroll
            for (int q = 0; q < NPL; ++q)
                u[q] = fmaf(-b.c, sqdist<DP>(y, tab + (r + 16 * q) * DP), b.K - sh);
            double gc = 0.0, mc = 0.0;
            // p = 0 .. m-1: label bits; p = m: the MI term (every point in subset 0).
#pragma unroll
            for (int p = 0; p <= m; ++p) {
                const bool want = p < m ? ((mask >> p) & 1u) != 0u : ((mask & kMiFlag) != 0u && b.tx != nullptr);
                if (__ballot(want) == 0ull) continue;
                // Far-only for a row that passed its near log-sum and the far side of the bit: the
                // far subset is summed under the fixed shift sh, all its terms being below 2^0.  A
                // sum of at least 2^-95 holds its largest term above 2^-102, so the terms flushed
                // below 2^-126 are under 2^-24 of the sum.  Every other row takes the two-pass path
                // below; each row's choice depends on its own symbol only, so the results do not
                // depend on which queue entries share a wavefront.
                bool far_ok = false;
                if (p < m && p < kFarBits && __ballot(want && has_near) != 0ull) {
                    const int fb = (int)((mask >> (kFarShift + p)) & 1u);
                    // all-ones when the far side is bit 1; opaque, so that the pick below stays a
                    // bit select (a select of the two registers by fb could be turned into a
                    // run-time index into u, which would put u in scratch memory)
                    uint32_t pick1 = 0u - (uint32_t)fb;
                    asm volatile("" : "+v"(pick1));
                    float sf = 0.0f;
                    if (p < 4) {
                        if (((r >> p) & 1) == fb) {
#pragma unroll
                            for (int q = 0; q < NPL; ++q) sf += hw_exp2(u[q]);
                        }
                    } else {
#pragma unroll
                        for (int q = 0; q < NPL; ++q) {
                            if (((q >> (p - 4)) & 1) == 0) {  // pair q with q | (1 << (p-4)); take the far one
                                const uint32_t v0 = __builtin_bit_cast(uint32_t, u[q]);
                                const uint32_t v1 = __builtin_bit_cast(uint32_t, u[q | (1 << (p - 4))]);
                                sf += hw_exp2(__builtin_bit_cast(float, (v1 & pick1) | (v0 & ~pick1)));
                            }
                        }
                    }
                    sf = row_reduce_f(sf, fadd2);
                    far_ok = has_near && sf >= 0x1p-95f;
                    if (want && far_ok && r == 0) {
                        // L = log2 S1 - log2 S0: the far log-sum exact, the near one passed
                        const float lf = sh + hw_log2(sf);
                        const float L = fb ? lf - near_lse : near_lse - lf;
                        if (b.llr) b.llr[(size_t)e.n * m + (m - 1 - p)] = L * 0.69314718055994531f;
                        if (b.tx) gc += (double)gmi_bit_term(L, (txl >> p) & 1);
                    }
                }
                if (__ballot(want && !far_ok) == 0ull) continue;
                // Two-pass log-sum-exp of both subsets: maxima, then sums under them.
                float mx0 = -INFINITY, mx1 = -INFINITY;
                if (p < 4) {
                    float mxl = u[0];
#pragma unroll
                    for (int q = 1; q < NPL; ++q) mxl = fmaxf(mxl, u[q]);
                    const bool one = ((r >> p) & 1) != 0;
                    mx0 = one ? -INFINITY : mxl;
                    mx1 = one ? mxl : -INFINITY;
                } else {
#pragma unroll
                    for (int q = 0; q < NPL; ++q) {
                        if (p < m && ((q >> (p - 4)) & 1)) mx1 = fmaxf(mx1, u[q]);
                        else mx0 = fmaxf(mx0, u[q]);
                    }
                }
                mx0 = row_reduce_f(mx0, fmax2);
                mx1 = row_reduce_f(mx1, fmax2);
                float s0 = 0.0f, s1 = 0.0f;
                if (p < 4) {
                    const bool one = ((r >> p) & 1) != 0;
                    const float sl_shift = one ? mx1 : mx0;
                    float sl = 0.0f;
#pragma unroll
                    for (int q = 0; q < NPL; ++q) sl += hw_exp2(u[q] - sl_shift);
                    s0 = one ? 0.0f : sl;
                    s1 = one ? sl : 0.0f;
                } else {
#pragma unroll
                    for (int q = 0; q < NPL; ++q) {
                        if (p < m && ((q >> (p - 4)) & 1)) s1 += hw_exp2(u[q] - mx1);
                        else s0 += hw_exp2(u[q] - mx0);
                    }
                }
                s0 = row_reduce_f(s0, fadd2);
                s1 = row_reduce_f(s1, fadd2);
                if (want && !far_ok && r == 0) {
                    if (p < m) {
                        const float L = (mx1 - mx0) + (hw_log2(s1) - hw_log2(s0));
                        if (b.llr) b.llr[(size_t)e.n * m + (m - 1 - p)] = L * 0.69314718055994531f;
                        if (b.tx) gc += (double)gmi_bit_term(L, (txl >> p) & 1);
                    } else {
                        const float lse_all = (mx0 + hw_log2(s0)) + sh;
                        const float ttx = fmaf(-b.c, sqdist<DP>(y, tab + txl * DP), b.K);
                        mc += (double)((float)m - (lse_all - ttx));
                    }
                }
            }
            if (live && r == 0) {
                add((int)e.tag, slot, 0, gc);
                add((int)e.tag, slot, 1, mc);
            }
        }
        __syncthreads();  // the chunk's entries are read before the next chunk overwrites them
    }
}

// Exclusive prefix of the queue regions' fill into s_qpre[0 .. kQueueRegions]: wave 0 of the
// block computes it; the caller synchronises the block before reading it.
__device__ __forceinline__ void queue_prefix(const Sinks& k, uint32_t* s_qpre) {
    static_assert(kQueueRegions == 64, "one wave scans the region counts");
    if (threadIdx.x < 64) {  // wave 0, fully active
        const int r = threadIdx.x;
        uint32_t x = min(k.queue_count[r * kQueueStride], k.queue_cap / kQueueRegions);
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t y = __shfl_up(x, off, 64);
            if (r >= off) x += y;
        }
        s_qpre[r + 1] = x;
        if (r == 0) s_qpre[0] = 0u;
    }
}

// Position in k.queue of entry i < s_qpre[kQueueRegions] of the filled regions read as one list:
// the largest region r with s_qpre[r] <= i holds it at offset i - s_qpre[r].
__device__ __forceinline__ size_t queue_index(const Sinks& k, const uint32_t* s_qpre, uint32_t i) {
    uint32_t r = 0;
#pragma unroll
    for (uint32_t step = kQueueRegions / 2; step >= 1; step >>= 1)
        if (s_qpre[r + step] <= i) r += step;
    return (size_t)r * (k.queue_cap / kQueueRegions) + (i - s_qpre[r]);
}

// Drain the fix-up queue: symbols of constellations with at most kFixLaneMaxM points are
// recomputed one per lane (fixup_one: cheaper than wave reductions for so few points), the
// others one per wavefront (fixup_wave).  view(e) gives the block of a queue entry; tl is the
// wave's LDS slice of cache_pts floats.  Corrections go to the fixed-point accumulators (slot = lane in the lane
// pass, wave % kAccSlots in the wave pass).  The filled parts of the queue regions are read as
// one list (entry i lies in the region whose prefix range holds i); every entry's flagged
// pairs are added to fix_pairs[tag] here.
constexpr int kFixLaneMaxM = 64;

template <int DP, typename ViewFn>
__device__ void drain_fix_queue(const Sinks& k, ViewFn view, float* tl, int cache_pts, int uniform_M = 0,
                                const float* uniform_table = nullptr) {
    // Corrections of blocks (tags) below kFixLdsTags are summed per workgroup in LDS, as the same
    // fixed-point integers acc_add uses (so the totals are unchanged and order-independent), and
    // flushed once per workgroup: per-entry global atomics were the fix-up's bottleneck.
    constexpr int kFixLdsTags = 64;
    __shared__ unsigned long long s_acc[kFixLdsTags * 2];
    __shared__ uint32_t s_pairs[kFixLdsTags];
    __shared__ uint32_t s_qpre[kQueueRegions + 1];  // exclusive prefix of the regions' fill
    for (int i = threadIdx.x; i < kFixLdsTags * 2; i += blockDim.x) s_acc[i] = 0ull;
    for (int i = threadIdx.x; i < kFixLdsTags; i += blockDim.x) s_pairs[i] = 0u;
    queue_prefix(k, s_qpre);
    __syncthreads();
    auto fetch = [&](uint32_t i) -> FixEntry { return k.queue[queue_index(k, s_qpre, i)]; };
    auto count_pairs = [&](const FixEntry& e) {
        if (!k.fix_pairs) return;
        const uint32_t c = (uint32_t)__popc(e.mask & 0xFFFFu);
        if (c == 0u) return;
        if (e.tag < (uint32_t)kFixLdsTags) atomicAdd(&s_pairs[e.tag], c);
        else atomicAdd(k.fix_pairs + e.tag, c);
    };
    auto add = [&](int tag, int slot, int which, double v) {
        if (!k.acc) return;
        if (tag < kFixLdsTags) {
            const long long q = __double2ll_rn(v * kFixScale);
            if (q != 0) atomicAdd(&s_acc[tag * 2 + which], (unsigned long long)q);
        } else {
            acc_add(k.acc, tag, slot, which, v);
        }
    };
    uint32_t count = s_qpre[kQueueRegions];
    const int lane = threadIdx.x & 63;
    const uint32_t wave = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const uint32_t nwaves = gridDim.x * (blockDim.x >> 6);
    if ((uniform_M == 128 || uniform_M == 256) && uniform_table) {  // one constellation: four symbols per wave
        if (uniform_M == 128) fix_rows<DP, 8>(k, view, add, fetch, count_pairs, count, uniform_table);
        else fix_rows<DP, 16>(k, view, add, fetch, count_pairs, count, uniform_table);
        count = 0;  // nothing left for the lane and wave passes
    }
    for (uint32_t base = wave * 64; base < count; base += nwaves * 64) {
        const uint32_t i = base + lane;
        if (i < count) {
            const FixEntry e = fetch(i);
            count_pairs(e);
            const BlockView b = view(e);
            if (b.M <= kFixLaneMaxM) {
                double gc = 0.0, mc = 0.0;
                fixup_one<DP>(b, k, e.n, e.mask, gc, mc);
                add((int)e.tag, lane, 0, gc);
                add((int)e.tag, lane, 1, mc);
            }
        }
    }
    const int slot = (int)(wave % kAccSlots);
    for (uint32_t i = wave; i < count; i += nwaves) {
        const FixEntry e = fetch(i);
        const BlockView b = view(e);
        if (b.M > kFixLaneMaxM) {
            double gc = 0.0, mc = 0.0;
            fixup_wave<DP>(b, k, e.n, e.mask, tl, cache_pts, gc, mc);
            if (lane == 0) {
                add((int)e.tag, slot, 0, gc);
                add((int)e.tag, slot, 1, mc);
            }
        }
    }
    __syncthreads();
    if (k.acc) {
        const int bslot = (int)(blockIdx.x % kAccSlots);
        for (int i = threadIdx.x; i < kFixLdsTags * 2; i += blockDim.x)
            if (s_acc[i] != 0ull) atomicAdd(k.acc + ((size_t)(i >> 1) * kAccSlots + bslot) * 2 + (i & 1), s_acc[i]);
    }
    if (k.fix_pairs)
        for (int i = threadIdx.x; i < kFixLdsTags; i += blockDim.x)
            if (s_pairs[i] != 0u) atomicAdd(k.fix_pairs + i, s_pairs[i]);
}

}  // namespace dm
