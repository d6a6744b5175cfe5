// Host-visible argument blocks and launchers of the learned-demapper kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dm {

enum : int { kEpiPartial = 0, kEpiFwdHidden = 1, kEpiFwdOut = 2, kEpiBwdHidden = 3 };

struct GemmArgs {
    const __bf16* A;    // M x K, row stride lda (elements)
    const __bf16* Bt;   // N x K, row stride ldb
    // Optional low words of A and Bt (same layouts): an operand carried as a BF16 pair
    // hi + lo (about 16 significant bits) contributes hi.b + lo.b (+ a.lo for the other side);
    // the lo.lo product is dropped (relative size 2^-16 of each product).
    const __bf16* A_lo;
    const __bf16* Bt_lo;
    int M, N, K, lda, ldb, splits, epi;
    float* part;        // PARTIAL: [splits][M][N]
    const float* bias;  // FWD_*: N
    float* Hout;        // FWD_HIDDEN: M x N pre-activations (ldh); FWD_OUT: outputs (optional)
    const float* Hin;   // BWD_HIDDEN: pre-activations (ldh)
    int ldh;
    __bf16* Aout;       // row-major output (ldo), may be null for BWD_HIDDEN
    __bf16* AoutT;      // transposed output (ldt)
    __bf16* Aout_lo;    // low words of the stored outputs, v - hi rounded to BF16 (may be null)
    __bf16* AoutT_lo;
    int ldo, ldt;
    const float* target;  // FWD_OUT: M x ld_target exact LLRs (nats)
    int ld_target, mout;
    float scale;          // FWD_OUT: 1 / (B m)
    float* loss_tiles;    // FWD_OUT: per-tile loss sums (may be null)
};

struct AdamArgs {
    float* w;
    float* m;
    float* v;
    const float* grad;
    __bf16* copy;   // may be null
    __bf16* copyT;  // may be null
    int rows, cols, mask_rows, mask_cols;
    float lr, beta1, beta2, eps, bc1, bc2;
};

// Inference: all BF16 weights staged in LDS; see mlp_infer.hip for the fragment layout.
struct MlpInferArgs {
    const uint4* frag;      // [W1 | W2 | W3] operand fragments
    const float* bias;      // b1 (256, unused: packed into the fragments) | b2 (256) | b3 (32, zero past m)
    const float* y;         // N x D received symbols
    const uint16_t* tx;     // N transmitted rows or null
    const uint16_t* row2label;
    float* llr;             // N x m or null
    int64_t N;
    int D, m, M;
    float snr_feature;      // (s - 7.5) / 7.5, s = -10 log10(2 sigma2)
    unsigned long long* acc;  // [kAccSlots][1] fixed-point GMI sum, or null
    uint32_t* bad_tx;
};

hipError_t launch_gemm_nt(const GemmArgs& g, hipStream_t st);
// Row sums of a BF16 matrix, with its low words Xlo (same layout) added when not null.
hipError_t launch_rowsum(const __bf16* X, const __bf16* Xlo, int rows, int cols, int ld, float* out, hipStream_t st);
hipError_t launch_reduce_splits(const float* part, int splits, size_t n, float* grad, hipStream_t st);
hipError_t launch_adam(const AdamArgs& a, hipStream_t st);
// Several parameter tensors in one launch: tensor k owns the flat elements [start[k], start[k+1]).
constexpr int kAdamMaxTensors = 8;
struct AdamBatch {
    AdamArgs t[kAdamMaxTensors];
    size_t start[kAdamMaxTensors + 1];
    int count;
};
hipError_t launch_adam_batch(const AdamBatch& b, hipStream_t st);
hipError_t launch_features(const float* y, const float* sigma2, int B, int D, __bf16* X, __bf16* Xt, hipStream_t st);

// Number of 16-byte fragments of the inference weight table (H = 256 hidden units).
size_t mlp_frag_count();
// Build the inference fragment table from the BF16 row-major (out x in) weights
// W1t [256 x 32] (D + 1 <= 14 inputs), W2t [256 x 256], W3t [32 x 256] and the FP32 bias b1.
hipError_t launch_mlp_pack(const __bf16* W1t, const __bf16* W2t, const __bf16* W3t, const float* b1, uint4* frag,
                           hipStream_t st);
hipError_t launch_mlp_infer(const MlpInferArgs& a, int grid, hipStream_t st);
hipError_t prepare_mlp_infer();

}  // namespace dm
