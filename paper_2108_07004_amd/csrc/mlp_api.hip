// C ABI of the learned demapper: an MLP (D+1) -> 256 -> 256 -> m trained on exact LLRs of a
// given constellation, run with an exact audit and per-SNR exact fallback.
//
// Device state of a network (H = 256), all owned by the dm_mlp object:
//   FP32 masters, Adam moments and gradients in one internal layout
//     W1t [256 x 32] (out x in, inputs >= D+1 stay zero) | b1 [256] | W2t [256 x 256] | b2 [256] |
//     W3t [32 x 256] (outputs >= m stay zero) | b3 [32]
//   BF16 copies rewritten by every Adam step: W1t, W2t, W3t (forward B operands) and W2, W3
//   (transposes, backward B operands); the inference fragment table and bias vector are
//   rebuilt from them lazily.
// The external weight order (host arrays) is the textbook one: W1 [(D+1) x 256] with
// out = x W + b, b1, W2 [256 x 256], b2, W3 [256 x m], b3 [m].
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <mutex>
#include <vector>

#include "api_internal.hpp"
#include "kernels.hpp"
#include "mlp_kernels.hpp"

namespace {

using dmapi::fail;
using dmapi::hip_fail;

constexpr int kH = 256;
constexpr size_t oW1 = 0, oB1 = oW1 + 256 * 32, oW2 = oB1 + 256, oB2 = oW2 + 256 * 256, oW3 = oB2 + 256,
                 oB3 = oW3 + 32 * 256, kMasterFloats = oB3 + 32;
constexpr int kLossHist = 64;                 // steps whose loss is kept for the reported mean
constexpr int64_t kTargetChunk = int64_t(1) << 20;  // samples per exact-target chunk
constexpr int kMaxBatch = 65536;

struct Ckpt {
    char magic[8];
    int32_t D, m, H, version;
    uint64_t hash;
    double snr_lo, snr_hi;
    int64_t step;
    int64_t n_floats;
};

}  // namespace

struct dm_mlp {
    int D = 0, m = 0, M = 0, device = 0, cus = 0;
    uint64_t hash = 0;
    double snr_lo = -std::numeric_limits<double>::infinity();
    double snr_hi = std::numeric_limits<double>::infinity();
    int64_t step = 0;
    float *w = nullptr, *mom = nullptr, *vel = nullptr, *grad = nullptr;  // kMasterFloats each
    __bf16 *W1t = nullptr, *W2t = nullptr, *W2 = nullptr, *W3t = nullptr, *W3 = nullptr;
    uint4* frag = nullptr;
    float* bias_inf = nullptr;  // b1 | b2 | b3 (32)
    bool frag_dirty = true;
    // batch scratch (grow-only)
    int B = 0;
    __bf16 *X = nullptr, *Xt = nullptr, *A1 = nullptr, *A1T = nullptr, *A2 = nullptr, *A2T = nullptr;
    __bf16 *dO = nullptr, *dOT = nullptr, *dH2 = nullptr, *dH2T = nullptr, *dH1T = nullptr;
    // Activations and deltas are BF16 pairs: each allocation above except X / Xt holds the hi
    // words, then the lo words (these pointers, into the same allocations).
    __bf16 *A1lo = nullptr, *A1Tlo = nullptr, *A2lo = nullptr, *A2Tlo = nullptr, *dOlo = nullptr, *dOTlo = nullptr;
    __bf16 *dH2lo = nullptr, *dH2Tlo = nullptr, *dH1Tlo = nullptr;
    float *H1 = nullptr, *H2 = nullptr, *part = nullptr, *loss_hist = nullptr;
    size_t part_floats = 0;
    float* targets = nullptr;
    int64_t target_rows = 0;
    unsigned long long* acc = nullptr;  // [n_snr][2][kAccSlots][2]
    uint32_t* bad = nullptr;
    int acc_snr = 0;
    void* h_stage = nullptr;
    size_t h_stage_bytes = 0;
    std::mutex mu;
};

namespace {

int64_t param_count(int D, int m) { return (int64_t)(D + 1) * kH + kH + (int64_t)kH * kH + kH + (int64_t)kH * m + m; }

template <class T>
int dev_alloc(T*& p, size_t count, const char* what) {
    if (p) {
        (void)hipFree(p);
        p = nullptr;
    }
    if (hipMalloc((void**)&p, std::max<size_t>(count, 1) * sizeof(T)) != hipSuccess) {
        (void)hipGetLastError();
        p = nullptr;
        return fail(DM_ENOMEM, "device allocation of %s (%zu bytes) failed", what, count * sizeof(T));
    }
    return DM_OK;
}

int host_stage(dm_mlp* n, size_t bytes) {
    if (n->h_stage_bytes >= bytes) return DM_OK;
    if (n->h_stage) (void)hipHostFree(n->h_stage);
    n->h_stage = nullptr;
    n->h_stage_bytes = 0;
    if (hipHostMalloc(&n->h_stage, bytes, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        return fail(DM_ENOMEM, "pinned staging allocation failed");
    }
    n->h_stage_bytes = bytes;
    return DM_OK;
}

// External (textbook) order -> internal layout, host side.
void to_internal(int D, int m, const float* ext, std::vector<float>& in) {
    in.assign(kMasterFloats, 0.0f);
    const float* p = ext;
    for (int i = 0; i < D + 1; ++i)
        for (int u = 0; u < kH; ++u) in[oW1 + (size_t)u * 32 + i] = *p++;
    for (int u = 0; u < kH; ++u) in[oB1 + u] = *p++;
    for (int i = 0; i < kH; ++i)
        for (int u = 0; u < kH; ++u) in[oW2 + (size_t)u * kH + i] = *p++;
    for (int u = 0; u < kH; ++u) in[oB2 + u] = *p++;
    for (int i = 0; i < kH; ++i)
        for (int o = 0; o < m; ++o) in[oW3 + (size_t)o * kH + i] = *p++;
    for (int o = 0; o < m; ++o) in[oB3 + o] = *p++;
}

void to_external(int D, int m, const std::vector<float>& in, float* ext) {
    float* p = ext;
    for (int i = 0; i < D + 1; ++i)
        for (int u = 0; u < kH; ++u) *p++ = in[oW1 + (size_t)u * 32 + i];
    for (int u = 0; u < kH; ++u) *p++ = in[oB1 + u];
    for (int i = 0; i < kH; ++i)
        for (int u = 0; u < kH; ++u) *p++ = in[oW2 + (size_t)u * kH + i];
    for (int u = 0; u < kH; ++u) *p++ = in[oB2 + u];
    for (int i = 0; i < kH; ++i)
        for (int o = 0; o < m; ++o) *p++ = in[oW3 + (size_t)o * kH + i];
    for (int o = 0; o < m; ++o) *p++ = in[oB3 + o];
}

// The six parameter tensors as Adam sees them (offsets into the internal layout).
struct Tensor {
    size_t off;
    int rows, cols, mask_rows, mask_cols;
    __bf16* copy;
    __bf16* copyT;
};

void tensors(const dm_mlp* n, Tensor t[6]) {
    t[0] = Tensor{oW1, 256, 32, 256, n->D + 1, n->W1t, nullptr};
    t[1] = Tensor{oB1, 1, 256, 1, 256, nullptr, nullptr};
    t[2] = Tensor{oW2, 256, 256, 256, 256, n->W2t, n->W2};
    t[3] = Tensor{oB2, 1, 256, 1, 256, nullptr, nullptr};
    t[4] = Tensor{oW3, 32, 256, n->m, 256, n->W3t, n->W3};
    t[5] = Tensor{oB3, 1, 32, 1, n->m, nullptr, nullptr};
}

// Adam step on every tensor (lr == 0 and mask_rows == 0: only rewrite the BF16 copies).
int adam_all(dm_mlp* n, bool update, float lr, float b1, float b2, float eps, double bc1, double bc2,
             hipStream_t st) {
    Tensor t[6];
    tensors(n, t);
    dm::AdamBatch batch;
    std::memset(&batch, 0, sizeof batch);
    batch.count = 6;
    for (int k = 0; k < 6; ++k) {
        const Tensor& x = t[k];
        dm::AdamArgs& a = batch.t[k];
        a.w = n->w + x.off;
        a.m = n->mom + x.off;
        a.v = n->vel + x.off;
        a.grad = n->grad + x.off;
        a.copy = x.copy;
        a.copyT = x.copyT;
        a.rows = x.rows;
        a.cols = x.cols;
        a.mask_rows = update ? x.mask_rows : 0;
        a.mask_cols = x.mask_cols;
        a.lr = lr;
        a.beta1 = b1;
        a.beta2 = b2;
        a.eps = eps;
        a.bc1 = (float)bc1;
        a.bc2 = (float)bc2;
        batch.start[k + 1] = batch.start[k] + (size_t)x.rows * x.cols;
    }
    DM_HIP_TRY(dm::launch_adam_batch(batch, st));
    n->frag_dirty = true;
    return DM_OK;
}

int ensure_batch(dm_mlp* n, int B) {
    if (n->B >= B) return DM_OK;
    const size_t b = (size_t)B;
    int r;
    n->B = 0;
    if ((r = dev_alloc(n->X, b * 16, "X")) || (r = dev_alloc(n->Xt, 32 * b, "Xt")) ||
        (r = dev_alloc(n->A1, 2 * b * kH, "A1")) || (r = dev_alloc(n->A1T, 2 * b * kH, "A1T")) ||
        (r = dev_alloc(n->A2, 2 * b * kH, "A2")) || (r = dev_alloc(n->A2T, 2 * b * kH, "A2T")) ||
        (r = dev_alloc(n->dO, 2 * b * 32, "dO")) || (r = dev_alloc(n->dOT, 2 * b * 32, "dOT")) ||
        (r = dev_alloc(n->dH2, 2 * b * kH, "dH2")) || (r = dev_alloc(n->dH2T, 2 * b * kH, "dH2T")) ||
        (r = dev_alloc(n->dH1T, 2 * b * kH, "dH1T")) || (r = dev_alloc(n->H1, b * kH, "H1")) ||
        (r = dev_alloc(n->H2, b * kH, "H2")) || (r = dev_alloc(n->loss_hist, (size_t)kLossHist * (b / 32), "loss")))
        return r;
    n->A1lo = n->A1 + b * kH;
    n->A1Tlo = n->A1T + b * kH;
    n->A2lo = n->A2 + b * kH;
    n->A2Tlo = n->A2T + b * kH;
    n->dOlo = n->dO + b * 32;
    n->dOTlo = n->dOT + b * 32;
    n->dH2lo = n->dH2 + b * kH;
    n->dH2Tlo = n->dH2T + b * kH;
    n->dH1Tlo = n->dH1T + b * kH;
    n->part_floats = std::max<size_t>(16 * 65536, 64 * 8192);
    if ((r = dev_alloc(n->part, n->part_floats, "split-K partials"))) return r;
    n->B = B;
    return DM_OK;
}

// Largest power-of-two split of K = B into chunks that are multiples of 16.
int k_splits(int B, int cap) {
    int s = cap;
    while (s > 1 && (B % s != 0 || (B / s) % 16 != 0)) s >>= 1;
    return s;
}

dm::GemmArgs gemm(const __bf16* A, int lda, const __bf16* Bt, int ldb, int M, int N, int K, int epi) {
    dm::GemmArgs g;
    std::memset(&g, 0, sizeof g);
    g.A = A;
    g.lda = lda;
    g.Bt = Bt;
    g.ldb = ldb;
    g.M = M;
    g.N = N;
    g.K = K;
    g.splits = 1;
    g.epi = epi;
    return g;
}

// Weight gradient C[M x N] = A[M x B] . Bt[N x B]^T (each operand with its optional low words),
// split over B, reduced into grad + off.
int weight_grad(dm_mlp* n, const __bf16* A, const __bf16* A_lo, const __bf16* Bt, const __bf16* Bt_lo, int M, int N,
                int B, int cap, size_t off, hipStream_t st) {
    dm::GemmArgs g = gemm(A, B, Bt, B, M, N, B, dm::kEpiPartial);
    g.A_lo = A_lo;
    g.Bt_lo = Bt_lo;
    g.splits = k_splits(B, cap);
    g.part = n->part;
    DM_HIP_TRY(dm::launch_gemm_nt(g, st));
    DM_HIP_TRY(dm::launch_reduce_splits(n->part, g.splits, (size_t)M * N, n->grad + off, st));
    return DM_OK;
}

// Forward + backward of one batch: gradients into n->grad, per-tile loss into loss_tiles.
int enqueue_grad(dm_mlp* n, int B, const float* y, const float* sigma2, const float* target, float* loss_tiles,
                 hipStream_t st) {
    DM_HIP_TRY(dm::launch_features(y, sigma2, B, n->D, n->X, n->Xt, st));
    // layer 1
    dm::GemmArgs g = gemm(n->X, 16, n->W1t, 32, B, kH, 16, dm::kEpiFwdHidden);
    g.bias = n->w + oB1;
    g.Hout = n->H1;
    g.ldh = kH;
    g.Aout = n->A1;
    g.Aout_lo = n->A1lo;
    g.ldo = kH;
    g.AoutT = n->A1T;
    g.AoutT_lo = n->A1Tlo;
    g.ldt = B;
    DM_HIP_TRY(dm::launch_gemm_nt(g, st));
    // layer 2
    g = gemm(n->A1, kH, n->W2t, kH, B, kH, kH, dm::kEpiFwdHidden);
    g.A_lo = n->A1lo;
    g.bias = n->w + oB2;
    g.Hout = n->H2;
    g.ldh = kH;
    g.Aout = n->A2;
    g.Aout_lo = n->A2lo;
    g.ldo = kH;
    g.AoutT = n->A2T;
    g.AoutT_lo = n->A2Tlo;
    g.ldt = B;
    DM_HIP_TRY(dm::launch_gemm_nt(g, st));
    // layer 3 + loss + output gradient
    g = gemm(n->A2, kH, n->W3t, kH, B, 32, kH, dm::kEpiFwdOut);
    g.A_lo = n->A2lo;
    g.bias = n->w + oB3;
    g.target = target;
    g.ld_target = n->m;
    g.mout = n->m;
    g.scale = (float)(1.0 / ((double)B * n->m));
    g.Aout = n->dO;
    g.Aout_lo = n->dOlo;
    g.ldo = 32;
    g.AoutT = n->dOT;
    g.AoutT_lo = n->dOTlo;
    g.ldt = B;
    g.loss_tiles = loss_tiles;
    DM_HIP_TRY(dm::launch_gemm_nt(g, st));
    int r;
    if ((r = weight_grad(n, n->dOT, n->dOTlo, n->A2T, n->A2Tlo, 32, kH, B, 64, oW3, st))) return r;
    DM_HIP_TRY(dm::launch_rowsum(n->dOT, n->dOTlo, 32, B, B, n->grad + oB3, st));
    // back through layer 3 and GELU 2
    g = gemm(n->dO, 32, n->W3, 32, B, kH, 32, dm::kEpiBwdHidden);
    g.A_lo = n->dOlo;
    g.Hin = n->H2;
    g.ldh = kH;
    g.Aout = n->dH2;
    g.Aout_lo = n->dH2lo;
    g.ldo = kH;
    g.AoutT = n->dH2T;
    g.AoutT_lo = n->dH2Tlo;
    g.ldt = B;
    DM_HIP_TRY(dm::launch_gemm_nt(g, st));
    if ((r = weight_grad(n, n->dH2T, n->dH2Tlo, n->A1T, n->A1Tlo, kH, kH, B, 16, oW2, st))) return r;
    DM_HIP_TRY(dm::launch_rowsum(n->dH2T, n->dH2Tlo, kH, B, B, n->grad + oB2, st));
    // back through layer 2 and GELU 1
    g = gemm(n->dH2, kH, n->W2, kH, B, kH, kH, dm::kEpiBwdHidden);
    g.A_lo = n->dH2lo;
    g.Hin = n->H1;
    g.ldh = kH;
    g.AoutT = n->dH1T;
    g.AoutT_lo = n->dH1Tlo;
    g.ldt = B;
    DM_HIP_TRY(dm::launch_gemm_nt(g, st));
    if ((r = weight_grad(n, n->dH1T, n->dH1Tlo, n->Xt, nullptr, kH, 32, B, 64, oW1, st))) return r;
    DM_HIP_TRY(dm::launch_rowsum(n->dH1T, n->dH1Tlo, kH, B, B, n->grad + oB1, st));
    return DM_OK;
}

int validate_batch(int B) {
    if (B < 256 || B > kMaxBatch || B % 256) return fail(DM_EINVAL, "batch %d must be a multiple of 256 in [256, %d]", B, kMaxBatch);
    return DM_OK;
}

int upload_weights(dm_mlp* n, const float* ext) {
    std::vector<float> in;
    to_internal(n->D, n->m, ext, in);
    for (size_t i = 0; i < in.size(); ++i)
        if (!std::isfinite(in[i])) return fail(DM_EINVAL, "weight %zu is not finite", i);
    DM_HIP_TRY(hipMemcpy(n->w, in.data(), kMasterFloats * sizeof(float), hipMemcpyHostToDevice));
    DM_HIP_TRY(hipMemset(n->mom, 0, kMasterFloats * sizeof(float)));
    DM_HIP_TRY(hipMemset(n->vel, 0, kMasterFloats * sizeof(float)));
    DM_HIP_TRY(hipMemset(n->grad, 0, kMasterFloats * sizeof(float)));
    n->step = 0;
    int r = adam_all(n, false, 0.0f, 0.9f, 0.999f, 1e-8f, 1.0, 1.0, nullptr);
    if (r) return r;
    DM_HIP_TRY(hipDeviceSynchronize());
    return DM_OK;
}

int ensure_packed(dm_mlp* n, hipStream_t st) {
    if (!n->frag_dirty) return DM_OK;
    DM_HIP_TRY(dm::launch_mlp_pack(n->W1t, n->W2t, n->W3t, n->w + oB1, n->frag, st));
    DM_HIP_TRY(hipMemcpyAsync(n->bias_inf, n->w + oB1, kH * sizeof(float), hipMemcpyDeviceToDevice, st));
    DM_HIP_TRY(hipMemcpyAsync(n->bias_inf + kH, n->w + oB2, kH * sizeof(float), hipMemcpyDeviceToDevice, st));
    DM_HIP_TRY(hipMemcpyAsync(n->bias_inf + 2 * kH, n->w + oB3, 32 * sizeof(float), hipMemcpyDeviceToDevice, st));
    n->frag_dirty = false;
    return DM_OK;
}

double snr_db_of(double sigma2) { return -10.0 * std::log10(2.0 * sigma2); }

}  // namespace

extern "C" {

int64_t dm_mlp_param_count(int32_t D, int32_t m) {
    if (D < 1 || D > 13 || m < 1 || m > 32) return DM_EINVAL;
    return param_count(D, m);
}

void dm_mlp_destroy(dm_mlp* n) {
    if (!n) return;
    for (void* p : {(void*)n->w, (void*)n->mom, (void*)n->vel, (void*)n->grad, (void*)n->W1t, (void*)n->W2t,
                    (void*)n->W2, (void*)n->W3t, (void*)n->W3, (void*)n->frag, (void*)n->bias_inf, (void*)n->X,
                    (void*)n->Xt, (void*)n->A1, (void*)n->A1T, (void*)n->A2, (void*)n->A2T, (void*)n->dO,
                    (void*)n->dOT, (void*)n->dH2, (void*)n->dH2T, (void*)n->dH1T, (void*)n->H1, (void*)n->H2,
                    (void*)n->part, (void*)n->loss_hist, (void*)n->targets, (void*)n->acc, (void*)n->bad})
        if (p) (void)hipFree(p);
    if (n->h_stage) (void)hipHostFree(n->h_stage);
    delete n;
}

int dm_mlp_create(const dm_constellation* c, const float* weights, dm_mlp** out) {
    dmapi::clear_error();
    if (!c || !weights || !out) return fail(DM_EINVAL, "null argument");
    *out = nullptr;
    if (c->D > 13) return fail(DM_EUNSUPPORTED, "the learned demapper supports D <= 13 (D=%d)", c->D);
    if (c->m > 32) return fail(DM_EUNSUPPORTED, "the learned demapper supports m <= 32");
    int r = dmapi::check_current_device(c);
    if (r) return r;
    auto* n = new (std::nothrow) dm_mlp();
    if (!n) return fail(DM_ENOMEM, "host allocation failed");
    n->D = c->D;
    n->m = c->m;
    n->M = c->M;
    n->device = c->device;
    n->cus = c->cus;
    n->hash = c->hash;
    if ((r = dev_alloc(n->w, kMasterFloats, "weights")) || (r = dev_alloc(n->mom, kMasterFloats, "Adam m")) ||
        (r = dev_alloc(n->vel, kMasterFloats, "Adam v")) || (r = dev_alloc(n->grad, kMasterFloats, "gradients")) ||
        (r = dev_alloc(n->W1t, 256 * 32, "W1t")) || (r = dev_alloc(n->W2t, 256 * 256, "W2t")) ||
        (r = dev_alloc(n->W2, 256 * 256, "W2")) || (r = dev_alloc(n->W3t, 32 * 256, "W3t")) ||
        (r = dev_alloc(n->W3, 256 * 32, "W3")) || (r = dev_alloc(n->frag, dm::mlp_frag_count(), "fragments")) ||
        (r = dev_alloc(n->bias_inf, 2 * kH + 32, "biases")) || (r = dev_alloc(n->bad, 1, "flag")) ||
        (r = upload_weights(n, weights))) {
        dm_mlp_destroy(n);
        return r;
    }
    hipError_t e = dm::prepare_mlp_infer();
    if (e != hipSuccess) {
        dm_mlp_destroy(n);
        return hip_fail(e, "inference kernel attributes");
    }
    *out = n;
    return DM_OK;
}

int dm_mlp_set_weights(dm_mlp* n, const float* weights) {
    dmapi::clear_error();
    if (!n || !weights) return fail(DM_EINVAL, "null argument");
    std::lock_guard<std::mutex> lock(n->mu);
    return upload_weights(n, weights);
}

int dm_mlp_get_weights(const dm_mlp* cn, float* weights) {
    dmapi::clear_error();
    if (!cn || !weights) return fail(DM_EINVAL, "null argument");
    auto* n = const_cast<dm_mlp*>(cn);
    std::lock_guard<std::mutex> lock(n->mu);
    std::vector<float> in(kMasterFloats);
    DM_HIP_TRY(hipDeviceSynchronize());
    DM_HIP_TRY(hipMemcpy(in.data(), n->w, kMasterFloats * sizeof(float), hipMemcpyDeviceToHost));
    to_external(n->D, n->m, in, weights);
    return DM_OK;
}

int dm_mlp_info(const dm_mlp* n, int64_t* steps, double* snr_lo_db, double* snr_hi_db) {
    dmapi::clear_error();
    if (!n) return fail(DM_EINVAL, "null argument");
    if (steps) *steps = n->step;
    if (snr_lo_db) *snr_lo_db = n->snr_lo;
    if (snr_hi_db) *snr_hi_db = n->snr_hi;
    return DM_OK;
}

int dm_mlp_gradients(dm_mlp* n, const float* y, const float* sigma2, const float* target, int32_t B, float* grads,
                     double* loss, void* stream) {
    dmapi::clear_error();
    if (!n || !y || !sigma2 || !target || !grads) return fail(DM_EINVAL, "null argument");
    int r = validate_batch(B);
    if (r) return r;
    if ((r = dmapi::check_device_ptr(y, "y", n->device)) || (r = dmapi::check_device_ptr(sigma2, "sigma2", n->device)) ||
        (r = dmapi::check_device_ptr(target, "target", n->device)))
        return r;
    std::lock_guard<std::mutex> lock(n->mu);
    hipStream_t st = (hipStream_t)stream;
    if ((r = ensure_batch(n, B))) return r;
    if ((r = enqueue_grad(n, B, y, sigma2, target, n->loss_hist, st))) return r;
    std::vector<float> in(kMasterFloats), lt(B / 32);
    DM_HIP_TRY(hipMemcpyAsync(in.data(), n->grad, kMasterFloats * sizeof(float), hipMemcpyDeviceToHost, st));
    DM_HIP_TRY(hipMemcpyAsync(lt.data(), n->loss_hist, lt.size() * sizeof(float), hipMemcpyDeviceToHost, st));
    DM_HIP_TRY(hipStreamSynchronize(st));
    to_external(n->D, n->m, in, grads);
    if (loss) {
        double s = 0.0;
        for (float v : lt) s += v;
        *loss = s / ((double)B * n->m);
    }
    return DM_OK;
}

int dm_mlp_train(dm_mlp* n, const dm_constellation* cc, const dm_train_config* cfg, const float* y,
                 const float* sigma2, int64_t N, double* loss, void* stream) {
    dmapi::clear_error();
    auto* c = const_cast<dm_constellation*>(cc);
    if (!n || !c || !cfg || !y || !sigma2) return fail(DM_EINVAL, "null argument");
    int r = validate_batch(cfg->batch);
    if (r) return r;
    if (cfg->epochs < 1) return fail(DM_EINVAL, "epochs=%d < 1", cfg->epochs);
    if (!(cfg->lr > 0.0f) || !(cfg->lr_final >= 0.0f) || !std::isfinite(cfg->lr) || !std::isfinite(cfg->lr_final))
        return fail(DM_EINVAL, "learning rates must be finite, lr > 0, lr_final >= 0");
    if (cfg->target_prec != DM_PREC_FP32 && cfg->target_prec != DM_PREC_BF16 && cfg->target_prec != DM_PREC_BF16X3)
        return fail(DM_EUNSUPPORTED, "target precision must be FP32, BF16 or BF16X3");
    if (!(cfg->snr_lo_db <= cfg->snr_hi_db)) return fail(DM_EINVAL, "snr_lo_db > snr_hi_db");
    if (c->hash != n->hash || c->D != n->D || c->m != n->m)
        return fail(DM_EINVAL, "the network was created for another constellation");
    if (N < 0 || N >= (int64_t(1) << 31)) return fail(DM_EINVAL, "N=%lld out of range", (long long)N);
    const int B = cfg->batch;
    const int64_t steps_per_epoch = N / B;
    if (steps_per_epoch < 1) return fail(DM_EINVAL, "N=%lld is smaller than one batch (%d)", (long long)N, B);
    if ((r = dmapi::check_device_ptr(y, "y", n->device)) || (r = dmapi::check_device_ptr(sigma2, "sigma2", n->device)))
        return r;
    const float b1 = cfg->beta1 > 0.0f ? cfg->beta1 : 0.9f;
    const float b2 = cfg->beta2 > 0.0f ? cfg->beta2 : 0.999f;
    const float eps = cfg->eps > 0.0f ? cfg->eps : 1e-8f;
    std::lock_guard<std::mutex> lock(n->mu);
    hipStream_t st = (hipStream_t)stream;
    if ((r = ensure_batch(n, B))) return r;
    const int64_t chunk = std::max<int64_t>(B, (kTargetChunk / B) * B);
    if (n->target_rows < chunk) {
        if ((r = dev_alloc(n->targets, (size_t)chunk * n->m, "targets"))) return r;
        n->target_rows = chunk;
    }
    const int64_t total = steps_per_epoch * cfg->epochs;
    const int64_t used = steps_per_epoch * B;
    int64_t t = 0;
    const int tiles = B / 32;
    for (int ep = 0; ep < cfg->epochs; ++ep) {
        for (int64_t c0 = 0; c0 < used; c0 += chunk) {
            const int64_t cn = std::min<int64_t>(chunk, used - c0);
            if ((r = dmapi::llr_var_run(c, sigma2 + c0, y + c0 * n->D, cn, n->targets, cfg->target_prec, st))) return r;
            for (int64_t b0 = 0; b0 < cn; b0 += B, ++t) {
                const int64_t s = c0 + b0;
                if ((r = enqueue_grad(n, B, y + s * n->D, sigma2 + s, n->targets + b0 * n->m,
                                      n->loss_hist + (size_t)(t % kLossHist) * tiles, st)))
                    return r;
                const double frac = total > 1 ? (double)t / (double)(total - 1) : 0.0;
                const double lr = cfg->lr_final + 0.5 * (cfg->lr - cfg->lr_final) * (1.0 + std::cos(3.14159265358979323846 * frac));
                ++n->step;
                const double bc1 = 1.0 - std::pow((double)b1, (double)n->step);
                const double bc2 = 1.0 - std::pow((double)b2, (double)n->step);
                if ((r = adam_all(n, true, (float)lr, b1, b2, eps, bc1, bc2, st))) return r;
            }
        }
    }
    n->snr_lo = cfg->snr_lo_db;
    n->snr_hi = cfg->snr_hi_db;
    const int kept = (int)std::min<int64_t>(total, kLossHist);
    std::vector<float> lt((size_t)kLossHist * tiles);
    DM_HIP_TRY(hipMemcpyAsync(lt.data(), n->loss_hist, lt.size() * sizeof(float), hipMemcpyDeviceToHost, st));
    DM_HIP_TRY(hipStreamSynchronize(st));
    if (loss) {
        double s = 0.0;
        for (int k = 0; k < kept; ++k)
            for (int i = 0; i < tiles; ++i) s += lt[(size_t)((t - 1 - k) % kLossHist) * tiles + i];
        *loss = s / ((double)kept * B * n->m);
    }
    return DM_OK;
}

int dm_demap_learned(dm_mlp* n, const dm_constellation* cc, int n_snr, const double* sigma2, const float* const* y,
                     const uint16_t* tx, int64_t N, float* const* llr, const dm_learned_opts* opts, double* gmi,
                     double* gmi_loss, int* used_fallback, void* stream) {
    dmapi::clear_error();
    auto* c = const_cast<dm_constellation*>(cc);
    if (!n || !c || !sigma2 || !y || !used_fallback) return fail(DM_EINVAL, "null argument");
    if (n_snr < 1) return fail(DM_EINVAL, "n_snr=%d < 1", n_snr);
    if (N < 0 || N >= (int64_t(1) << 31)) return fail(DM_EINVAL, "N=%lld out of range", (long long)N);
    if (tx && !gmi) return fail(DM_EINVAL, "gmi output is required when tx is given");
    dm_learned_opts o{0.01, 6, DM_PREC_FP32};
    if (opts) o = *opts;
    if (o.audit_log2 < 0 || o.audit_log2 > 20) return fail(DM_EINVAL, "audit_log2=%d outside [0, 20]", o.audit_log2);
    if (o.exact_prec < DM_PREC_FP32 || o.exact_prec > DM_PREC_FP16X3) return fail(DM_EINVAL, "unknown precision %d", o.exact_prec);
    int r;
    for (int s = 0; s < n_snr; ++s)
        if ((r = dmapi::validate_sigma2(sigma2[s]))) return r;
    if (N == 0) {
        for (int s = 0; s < n_snr; ++s) {
            if (gmi) gmi[s] = NAN;
            if (gmi_loss) gmi_loss[s] = NAN;
            used_fallback[s] = DM_LEARNED_OK;
        }
        return DM_OK;
    }
    if ((r = dmapi::check_current_device(c))) return r;
    if (tx && (r = dmapi::check_device_ptr(tx, "tx", c->device))) return r;
    for (int s = 0; s < n_snr; ++s) {
        if ((r = dmapi::check_device_ptr(y[s], "y[s]", c->device))) return r;
        if (llr && (r = dmapi::check_device_ptr(llr[s], "llr[s]", c->device))) return r;
    }
    std::lock_guard<std::mutex> lock(n->mu);
    hipStream_t st = (hipStream_t)stream;
    const bool same = c->hash == n->hash && c->D == n->D && c->m == n->m;
    // 1. which SNR points the network covers
    std::vector<int> code(n_snr, DM_LEARNED_OK);
    for (int s = 0; s < n_snr; ++s) {
        const double sd = snr_db_of(sigma2[s]);
        if (!same) code[s] = DM_FALLBACK_CONSTELLATION;
        else if (!(sd >= n->snr_lo - 1e-9 && sd <= n->snr_hi + 1e-9)) code[s] = DM_FALLBACK_SNR;
    }
    const bool audit = tx && o.max_gmi_loss >= 0.0;
    const int64_t na = audit ? std::min<int64_t>(N, std::max<int64_t>((N + (int64_t(1) << o.audit_log2) - 1) >> o.audit_log2, 8192)) : 0;
    // 2. the network on the audit prefix [0, na) of every covered point (accumulator set 0); the
    //    rest [na, N) runs only for the points that pass (set 1), so a failed audit costs 1/64.
    if (n->acc_snr < n_snr) {
        if ((r = dev_alloc(n->acc, (size_t)n_snr * 2 * dm::kAccSlots * 2, "GMI accumulators"))) return r;
        n->acc_snr = n_snr;
    }
    const size_t acc_words = (size_t)n_snr * 2 * dm::kAccSlots * 2;
    if ((r = host_stage(n, acc_words * sizeof(unsigned long long) + 64))) return r;
    if ((r = ensure_packed(n, st))) return r;
    DM_HIP_TRY(hipMemsetAsync(n->acc, 0, acc_words * sizeof(unsigned long long), st));
    DM_HIP_TRY(hipMemsetAsync(n->bad, 0, sizeof(uint32_t), st));
    auto infer = [&](int s, int64_t lo, int64_t hi, int set) -> int {
        const int64_t cnt = hi - lo;
        if (cnt <= 0) return DM_OK;
        dm::MlpInferArgs a;
        std::memset(&a, 0, sizeof a);
        a.frag = n->frag;
        a.bias = n->bias_inf;
        a.row2label = c->d_row2label;
        a.D = n->D;
        a.m = n->m;
        a.M = c->M;
        a.snr_feature = (float)((snr_db_of(sigma2[s]) - 7.5) / 7.5);
        a.bad_tx = tx ? n->bad : nullptr;
        a.y = y[s] + lo * n->D;
        a.tx = tx ? tx + lo : nullptr;
        a.llr = llr ? llr[s] + lo * n->m : nullptr;
        a.N = cnt;
        a.acc = tx ? n->acc + ((size_t)s * 2 + set) * dm::kAccSlots * 2 : nullptr;
        const int64_t tiles = (cnt + 31) / 32;
        const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((tiles + 7) / 8, n->cus));
        DM_HIP_TRY(dm::launch_mlp_infer(a, grid, st));
        return DM_OK;
    };
    auto* acc_h = (unsigned long long*)n->h_stage;
    auto* bad_h = (uint32_t*)(acc_h + acc_words);
    auto slot_sum = [&](int s, int set) {
        long long v = 0;
        for (int k = 0; k < dm::kAccSlots; ++k) v += (long long)acc_h[(((size_t)s * 2 + set) * dm::kAccSlots + k) * 2];
        return (double)v / dm::kFixScale;
    };
    for (int s = 0; s < n_snr; ++s) {
        if (gmi_loss) gmi_loss[s] = NAN;
        if (code[s] == DM_LEARNED_OK && audit && (r = infer(s, 0, na, 0))) return r;
    }
    // 3. exact audit of the prefixes (one launch over all audited points; synchronises)
    std::vector<int> aud;
    for (int s = 0; s < n_snr; ++s)
        if (code[s] == DM_LEARNED_OK && audit) aud.push_back(s);
    if (!aud.empty()) {
        DM_HIP_TRY(hipMemcpyAsync(acc_h, n->acc, acc_words * sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
        DM_HIP_TRY(hipMemcpyAsync(bad_h, n->bad, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
        std::vector<double> s2, g(aud.size());
        std::vector<const float*> ys;
        for (int s : aud) {
            s2.push_back(sigma2[s]);
            ys.push_back(y[s]);
        }
        if ((r = dmapi::gmi_run(c, (int)aud.size(), s2.data(), ys.data(), tx, na, nullptr, g.data(), nullptr,
                                o.exact_prec, st)))
            return r;
        if (*bad_h) return fail(DM_EINVAL, "a transmitted index is >= M");
        for (size_t i = 0; i < aud.size(); ++i) {
            const int s = aud[i];
            const double loss_est = g[i] - slot_sum(s, 0) / (double)na;
            if (gmi_loss) gmi_loss[s] = loss_est;
            if (loss_est > o.max_gmi_loss) code[s] = DM_FALLBACK_AUDIT;
        }
    }
    // 4. the network on the rest of every point it keeps; exact over whole blocks elsewhere
    for (int s = 0; s < n_snr; ++s)
        if (code[s] == DM_LEARNED_OK && (r = infer(s, audit ? na : 0, N, 1))) return r;
    DM_HIP_TRY(hipMemcpyAsync(acc_h, n->acc, acc_words * sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
    DM_HIP_TRY(hipMemcpyAsync(bad_h, n->bad, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    DM_HIP_TRY(hipStreamSynchronize(st));
    if (tx && *bad_h) return fail(DM_EINVAL, "a transmitted index is >= M");
    std::vector<int> exact_pts;
    for (int s = 0; s < n_snr; ++s) {
        if (code[s] == DM_LEARNED_OK) {
            if (tx) gmi[s] = (slot_sum(s, 0) + slot_sum(s, 1)) / (double)N;
        } else {
            exact_pts.push_back(s);
        }
    }
    if (!exact_pts.empty()) {
        std::vector<double> s2, g(exact_pts.size());
        std::vector<const float*> ys;
        std::vector<float*> ls;
        for (int s : exact_pts) {
            s2.push_back(sigma2[s]);
            ys.push_back(y[s]);
            if (llr) ls.push_back(llr[s]);
        }
        if (tx) {
            if ((r = dmapi::gmi_run(c, (int)exact_pts.size(), s2.data(), ys.data(), tx, N, llr ? ls.data() : nullptr,
                                    g.data(), nullptr, o.exact_prec, st)))
                return r;
            for (size_t i = 0; i < exact_pts.size(); ++i) gmi[exact_pts[i]] = g[i];
        } else if (llr) {
            for (size_t i = 0; i < exact_pts.size(); ++i)
                if ((r = dm_demap_llr(c, s2[i], ys[i], N, ls[i], o.exact_prec, stream))) return r;
            DM_HIP_TRY(hipStreamSynchronize(st));
        }
    }
    for (int s = 0; s < n_snr; ++s) used_fallback[s] = code[s];
    return DM_OK;
}

int dm_mlp_save(const dm_mlp* cn, const char* path) {
    dmapi::clear_error();
    if (!cn || !path) return fail(DM_EINVAL, "null argument");
    auto* n = const_cast<dm_mlp*>(cn);
    std::lock_guard<std::mutex> lock(n->mu);
    std::vector<float> buf(3 * kMasterFloats);
    DM_HIP_TRY(hipDeviceSynchronize());
    DM_HIP_TRY(hipMemcpy(buf.data(), n->w, kMasterFloats * sizeof(float), hipMemcpyDeviceToHost));
    DM_HIP_TRY(hipMemcpy(buf.data() + kMasterFloats, n->mom, kMasterFloats * sizeof(float), hipMemcpyDeviceToHost));
    DM_HIP_TRY(hipMemcpy(buf.data() + 2 * kMasterFloats, n->vel, kMasterFloats * sizeof(float), hipMemcpyDeviceToHost));
    Ckpt h;
    std::memset(&h, 0, sizeof h);
    std::memcpy(h.magic, "DMMLPCK1", 8);
    h.D = n->D;
    h.m = n->m;
    h.H = kH;
    h.version = 1;
    h.hash = n->hash;
    h.snr_lo = n->snr_lo;
    h.snr_hi = n->snr_hi;
    h.step = n->step;
    h.n_floats = (int64_t)buf.size();
    FILE* f = std::fopen(path, "wb");
    if (!f) return fail(DM_EINVAL, "cannot open %s for writing", path);
    const bool ok = std::fwrite(&h, sizeof h, 1, f) == 1 && std::fwrite(buf.data(), sizeof(float), buf.size(), f) == buf.size();
    const bool closed = std::fclose(f) == 0;
    if (!ok || !closed) return fail(DM_EINVAL, "short write to %s", path);
    return DM_OK;
}

int dm_mlp_load(const dm_constellation* c, const char* path, dm_mlp** out) {
    dmapi::clear_error();
    if (!c || !path || !out) return fail(DM_EINVAL, "null argument");
    *out = nullptr;
    FILE* f = std::fopen(path, "rb");
    if (!f) return fail(DM_EINVAL, "cannot open %s", path);
    Ckpt h;
    std::vector<float> buf(3 * kMasterFloats);
    bool ok = std::fread(&h, sizeof h, 1, f) == 1;
    ok = ok && std::memcmp(h.magic, "DMMLPCK1", 8) == 0 && h.version == 1 && h.H == kH &&
         h.n_floats == (int64_t)buf.size();
    ok = ok && std::fread(buf.data(), sizeof(float), buf.size(), f) == buf.size();
    std::fclose(f);
    if (!ok) return fail(DM_EINVAL, "%s is not a learned-demapper checkpoint of this version", path);
    if (h.D != c->D || h.m != c->m)
        return fail(DM_EINVAL, "checkpoint shape (D=%d, m=%d) does not match the constellation", h.D, h.m);
    std::vector<float> ext((size_t)param_count(h.D, h.m));
    to_external(h.D, h.m, std::vector<float>(buf.begin(), buf.begin() + kMasterFloats), ext.data());
    dm_mlp* n = nullptr;
    int r = dm_mlp_create(c, ext.data(), &n);
    if (r) return r;
    hipError_t e = hipMemcpy(n->w, buf.data(), kMasterFloats * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(n->mom, buf.data() + kMasterFloats, kMasterFloats * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(n->vel, buf.data() + 2 * kMasterFloats, kMasterFloats * sizeof(float), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        dm_mlp_destroy(n);
        return hip_fail(e, "checkpoint upload");
    }
    n->hash = h.hash;
    n->snr_lo = h.snr_lo;
    n->snr_hi = h.snr_hi;
    n->step = h.step;
    *out = n;
    return DM_OK;
}

}  // extern "C"
