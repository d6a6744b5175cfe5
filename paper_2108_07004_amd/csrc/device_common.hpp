// Device-side helpers and launch-argument layout shared by the demapping kernels (gfx950).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dm {

constexpr int kMaxSnrPerLaunch = 32;  // SNR points per launch (kernel-argument block stays < 1 KiB)
constexpr int kAccSlots = 64;         // fixed-point accumulator slots per block (spreads atomics)
constexpr double kFixScale = 268435456.0;  // 2^28: GMI/MI sums are accumulated as int64 * 2^-28
constexpr uint32_t kMiFlag = 0x80000000u;  // fix-up mask bit: recompute the MI term
constexpr int kFarShift = 16;  // fix-up mask bit kFarShift + p: bit p's far subset is its bit-1 side
constexpr int kFarBits = 15;   // label bits p < kFarBits carry that side (bits 16..30 of the mask)

// Fix-up mask of a flagged label bit p with subset sums s0 / s1 (the far side: the smaller).
__device__ __forceinline__ uint32_t flag_bits(int p, float s0, float s1) {
    return (1u << p) | ((p < kFarBits && s1 < s0) ? 1u << (kFarShift + p) : 0u);
}

// The fix-up queue is split into kQueueRegions equal regions, each with its own counter
// (kQueueStride words apart): a wave appends to the region its global wave index hashes to.
// Device-scope atomics on one address serialise at ~11 ns each on MI355X (measured), and at high
// SNR nearly every 32-symbol batch queues symbols, so a single counter made the queue, not the
// arithmetic, the bound of those launches; 64 counters spread the same atomics ~35x thinner.
constexpr int kQueueRegions = 64;
constexpr int kQueueStride = 64;                                   // words between two counters
constexpr int kQueueCounterWords = kQueueRegions * kQueueStride;  // counter array, zeroed per launch
constexpr int kFixCached = 2048;  // the wave fix-up caches a symbol's exponents in LDS up to this M

// One symbol whose far-subset sums underflowed the shared exponent window.
struct FixEntry {
    uint32_t n;     // symbol index within its block
    uint32_t tag;   // block (SNR point or instance) the symbol belongs to
    uint32_t mask;  // bit p set: recompute label bit p (p < 16); kMiFlag: recompute the MI term;
                    // bit kFarShift + p: bit p's far (underflowed) subset is the bit-1 side
    uint32_t near;  // bits of log2 of the symbol's total sum (t units) when that total is at least
                    // 2^(m-78) and finite (kNearNone otherwise): then a flagged bit's near subset
                    // holds all of it to FP32 precision, and only its far subset needs recomputing
};
constexpr uint32_t kNearNone = 0x7FC00000u;  // quiet NaN: no near-subset log-sum passed

// The FixEntry.near word for a symbol total stot (the demapper's own sum of all M terms).
__device__ __forceinline__ uint32_t near_word(float stot, int m, bool bad) {
    if (bad || !(stot >= __builtin_ldexpf(1.0f, m - 78)) || !(stot < 3.0e38f)) return kNearNone;
    const int e = __builtin_amdgcn_frexp_expf(stot);
    const float l = (float)e + __builtin_amdgcn_logf(__builtin_amdgcn_frexp_mantf(stot));
    return __builtin_bit_cast(uint32_t, l);
}

// One received block: a constellation at one noise level with its data.
struct BlockView {
    const float* table;          // M x DP FP32 points in label order (row j has label j)
    const uint16_t* row2label;   // M: label of each caller row
    const uint16_t* tx;          // N transmitted caller rows, or null (no GMI/MI)
    const float* y;              // N x D received symbols
    float* llr;                  // N x m output or null
    int64_t N;
    int32_t M, D, m;
    float c;                     // log2(e) / (2 sigma2), rounded once from FP64
    float K;                     // exponent offset: e_j = 2^(K - c ||y - x_j||^2)
    float flag_thresh;           // 2^(m-102): a subset sum below this is recomputed
    float near_thresh;           // 2^(m-42): GMI-only shortcut bound for the near subset
    int32_t want_llr;
    int32_t tag;                 // accumulator row and fix-up tag of this block
};

// Where kernels put results shared across blocks.
struct Sinks {
    unsigned long long* acc;     // [tags][kAccSlots][2] int64 fixed-point GMI / MI sums, or null
    uint32_t* fix_pairs;         // [tags] count of (symbol, bit) pairs sent to the fix-up, or null
    uint32_t* bad_tx;            // set to 1 when a transmitted index is >= M (clamped, reported)
    FixEntry* queue;             // queue_cap entries: kQueueRegions regions of queue_cap / kQueueRegions
    uint32_t* queue_count;       // kQueueCounterWords: region r's counter at word r * kQueueStride
    uint32_t queue_cap;
};

struct SnrArg {
    const float* y;  // N x D received block
    float* llr;      // N x m output or null
    float c;         // log2(e) / (2 sigma2)
    int32_t pad;
};

// Hard-decision launch over up to kMaxSnrPerLaunch received blocks of one transmitted block.
struct HardArgs {
    const float* table;          // M x DP, label order
    const uint16_t* row2label;   // M
    const uint16_t* tx;          // N transmitted rows (with counts)
    const float* y[kMaxSnrPerLaunch];
    uint16_t* labels_out[kMaxSnrPerLaunch];  // decided labels per block, or null
    int64_t N, tiles_per_blk;
    int M, D, n_blk;
    unsigned long long* counts;  // [n_blk][2]: symbol errors, bit errors; null = no counting
    uint32_t* bad_tx;
};

// Multi-SNR launch over one constellation and one transmitted block.
struct LaunchArgs {
    const float* table;
    const uint16_t* row2label;
    const uint16_t* tx;
    int64_t N;
    int64_t tiles_per_snr;
    int32_t M, D, m, n_snr;
    float K, flag_thresh, near_thresh;
    int32_t want_llr;
    const float* sigma2_sym;     // per-symbol noise variances (overrides snr[].c), or null
    Sinks sinks;
    SnrArg snr[kMaxSnrPerLaunch];
};

// ---- batched launch over many instances ----
constexpr int kKindValu = 0;  // FP32 direct-difference body
constexpr int kKindMfma = 1;  // MFMA cross-term body
constexpr int kBatchedLdsBytes = 131072;  // largest staged table (FP32 rows or MFMA fragments)
// Dynamic LDS of the batched kernel: the table plus the one 2 KiB fragment tile (split
// operands) that the MFMA pipeline reads past a 16-tile block.
constexpr int kBatchedLdsAlloc = kBatchedLdsBytes + 2048;

struct BatchDesc {             // one instance (device memory); view.tag = instance index
    BlockView view;            // table: FP32 label order with row stride 8
    const uint4* frag;         // MFMA point operands, fragment order (D padded to 8), or null
    const uint16_t* pv;        // the same operands per label, or null
    int32_t kind;
    int32_t sub;               // symbol tiles per work item (work item = sub x the body's tile)
};

struct WorkItem {              // symbols [n0, n0 + tile) of one instance
    int32_t inst;
    int32_t pad;
    int64_t n0;
};

struct BatchArgs {
    const BatchDesc* desc;
    const WorkItem* items;     // instance by instance, largest instance cost first
    int32_t n_items;
    int32_t grab;              // items per claim; claims start at multiples of grab
    uint32_t* next;            // claim counter (zeroed before every launch)
    Sinks sinks;
};

__device__ __forceinline__ BlockView view_snr(const LaunchArgs& a, int s) {
    BlockView v;
    v.table = a.table;
    v.row2label = a.row2label;
    v.tx = a.tx;
    v.y = a.snr[s].y;
    v.llr = a.snr[s].llr;
    v.N = a.N;
    v.M = a.M;
    v.D = a.D;
    v.m = a.m;
    v.c = a.snr[s].c;
    v.K = a.K;
    v.flag_thresh = a.flag_thresh;
    v.near_thresh = a.near_thresh;
    v.want_llr = a.want_llr;
    v.tag = s;
    return v;
}

// View of SNR block s as seen by symbol n (per-symbol noise variance when given).
__device__ __forceinline__ BlockView view_sym(const LaunchArgs& a, int s, int64_t n, bool active) {
    BlockView v = view_snr(a, s);
    if (a.sigma2_sym) v.c = 0.72134752044448170f / (active ? a.sigma2_sym[n] : 1.0f);  // log2(e) / (2 sigma2)
    return v;
}

// Label of the transmitted row; an out-of-range row is clamped and reported.
__device__ __forceinline__ int tx_label(const BlockView& b, const Sinks& k, int64_t n) {
    uint32_t r = b.tx[n];
    if (r >= (uint32_t)b.M) {
        if (k.bad_tx) atomicOr(k.bad_tx, 1u);
        r = 0;
    }
    return (int)b.row2label[r];
}

__device__ __forceinline__ float hw_exp2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ float hw_log2(float x) { return __builtin_amdgcn_logf(x); }

// log2(a) - log2(b) with exact binary exponents: the mantissa logs are O(1), so the
// result keeps FP32 accuracy even when both logs are ~100 (the exponent offset K).
__device__ __forceinline__ float log2_ratio(float a, float b) {
    const int ea = __builtin_amdgcn_frexp_expf(a);
    const int eb = __builtin_amdgcn_frexp_expf(b);
    const float ma = __builtin_amdgcn_frexp_mantf(a);
    const float mb = __builtin_amdgcn_frexp_mantf(b);
    return (float)(ea - eb) + (hw_log2(ma) - hw_log2(mb));
}

// log2(1 + u) for u in [0, 1]; the series branch keeps the tiny-u tail that 1+u would lose.
__device__ __forceinline__ float log2_1p(float u) {
    return (u < 0x1p-12f) ? u * (1.44269504088896341f - 0.72134752044448170f * u) : hw_log2(1.0f + u);
}

// Per-bit GMI term 1 - log2(1 + 2^(s L)), L the LLR in log2 units, s = +1 for a
// transmitted 0 and -1 for a transmitted 1.
__device__ __forceinline__ float gmi_bit_term(float L, int tx_bit) {
    const float x = tx_bit ? -L : L;
    return 1.0f - (fmaxf(x, 0.0f) + log2_1p(hw_exp2(-fabsf(x))));
}

// LLR in log2 units and the per-bit GMI term from the two subset sums (positive, normal):
// L = log2 s1 - log2 s0 and g = 1 - log2(S / s_b), s_b the transmitted bit's sum and S the
// symbol's total (the same for every bit: s0 + s1 = S), whose binary exponent es and mantissa
// log ls the caller forms once per symbol.  Both use the exact binary exponents and O(1)
// mantissa logs, so the GMI term needs no exp2: when s_b dominates, S and s_b share their
// exponent and the mantissa logs differ by the small true value.
__device__ __forceinline__ float llr_gmi(float s0, float s1, int tx_bit, int es, float ls, float& g) {
    const int e0 = __builtin_amdgcn_frexp_expf(s0), e1 = __builtin_amdgcn_frexp_expf(s1);
    const float l0 = hw_log2(__builtin_amdgcn_frexp_mantf(s0)), l1 = hw_log2(__builtin_amdgcn_frexp_mantf(s1));
    const int eb = tx_bit ? e1 : e0;
    const float lb = tx_bit ? l1 : l0;
    g = 1.0f - ((float)(es - eb) + (ls - lb));
    return (float)(e1 - e0) + (l1 - l0);
}

// Butterfly sum over the 64 lanes of a wavefront, FP64, fixed order (every lane gets the sum).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ void acc_add(unsigned long long* acc, int snr, int slot, int which, double v) {
    const long long q = __double2ll_rn(v * kFixScale);
    if (q != 0) atomicAdd(acc + ((size_t)snr * kAccSlots + slot) * 2 + which, (unsigned long long)q);
}

// Direct squared distance ||y - x||^2 in FP32 (differences first, then squares).
template <int D>
__device__ __forceinline__ float sqdist(const float (&y)[D], const float* x) {
    float acc = 0.0f;
#pragma unroll
    for (int d = 0; d < D; ++d) {
        const float t = y[d] - x[d];
        acc = fmaf(t, t, acc);
    }
    return acc;
}

// ---- exact recomputation shared by every demapping kernel (far-subset fix-up) ----

template <int DP>
__device__ __forceinline__ void load_symbol(float (&y)[DP], const float* src, int D, bool active) {
#pragma unroll
    for (int d = 0; d < DP; ++d) y[d] = (active && d < D) ? src[d] : 0.0f;
}

// Exact log-sum-exp (log2 units, t_j = K - c d_j^2) of the subsets of label bit p,
// with each subset shifted by its own maximum.  Returns L = log2 S^1 - log2 S^0.
template <int DP>
__device__ float exact_bit_llr2(const float (&y)[DP], const float* table, int M, int p, float c, float K) {
    float mx0 = -INFINITY, mx1 = -INFINITY;
    for (int j = 0; j < M; ++j) {
        const float t = fmaf(-c, sqdist<DP>(y, table + (size_t)j * DP), K);
        if ((j >> p) & 1) mx1 = fmaxf(mx1, t);
        else mx0 = fmaxf(mx0, t);
    }
    float s0 = 0.0f, s1 = 0.0f;
    for (int j = 0; j < M; ++j) {
        const float t = fmaf(-c, sqdist<DP>(y, table + (size_t)j * DP), K);
        if ((j >> p) & 1) s1 += hw_exp2(t - mx1);
        else s0 += hw_exp2(t - mx0);
    }
    return (mx1 - mx0) + (hw_log2(s1) - hw_log2(s0));
}

// MI term m - log2 sum_j 2^(t_j - t_tx), exact max shift.
template <int DP>
__device__ float exact_mi_term(const float (&y)[DP], const float* table, int M, int m, int txl, float c, float K) {
    float mx = -INFINITY;
    for (int j = 0; j < M; ++j) mx = fmaxf(mx, fmaf(-c, sqdist<DP>(y, table + (size_t)j * DP), K));
    float s = 0.0f;
    for (int j = 0; j < M; ++j) s += hw_exp2(fmaf(-c, sqdist<DP>(y, table + (size_t)j * DP), K) - mx);
    const float ttx = fmaf(-c, sqdist<DP>(y, table + (size_t)txl * DP), K);
    return (float)m - ((mx - ttx) + hw_log2(s));
}

// Recompute the flagged bits of one symbol in one lane; returns the GMI / MI corrections.
template <int DP>
__device__ void fixup_one(const BlockView& b, const Sinks& k, uint32_t n, uint32_t mask, double& gcorr,
                          double& mcorr) {
    float y[DP];
    load_symbol<DP>(y, b.y + (size_t)n * b.D, b.D, true);
    const int txl = b.tx ? tx_label(b, k, n) : 0;
    for (int p = 0; p < b.m; ++p) {
        if (!((mask >> p) & 1u)) continue;
        const float L = exact_bit_llr2<DP>(y, b.table, b.M, p, b.c, b.K);
        if (b.llr) b.llr[(size_t)n * b.m + (b.m - 1 - p)] = L * 0.69314718055994531f;
        if (b.tx) gcorr += (double)gmi_bit_term(L, (txl >> p) & 1);
    }
    if ((mask & kMiFlag) && b.tx) mcorr += (double)exact_mi_term<DP>(y, b.table, b.M, b.m, txl, b.c, b.K);
}

// Queue region of the calling wave (wave-uniform, so the compiler folds the lanes' counter
// increments into one atomic per wave).
__device__ __forceinline__ uint32_t queue_region() {
    const uint32_t w = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)(w % kQueueRegions));
}

// Queue a symbol for the fix-up (near: FixEntry.near of the symbol) in the wave's region; when
// that region is full the calling lane recomputes the symbol in place (slow but exact), counts
// its pairs, and the corrections come back through gc / mc.  Queued pairs are counted by the
// fix-up when it drains them.
template <int DP>
__device__ __forceinline__ void queue_or_fix(const BlockView& b, const Sinks& k, uint32_t n, uint32_t mask,
                                             uint32_t near, double& gc, double& mc) {
    const uint32_t seg = k.queue_cap / kQueueRegions;
    const uint32_t r = queue_region();
    const uint32_t slot = atomicAdd(k.queue_count + r * kQueueStride, 1u);
    if (slot < seg) {
        k.queue[(size_t)r * seg + slot] = FixEntry{n, (uint32_t)b.tag, mask, near};
    } else {
        if (k.fix_pairs) atomicAdd(k.fix_pairs + b.tag, (uint32_t)__popc(mask & 0xFFFFu));
        fixup_one<DP>(b, k, n, mask, gc, mc);
    }
}

}  // namespace dm
