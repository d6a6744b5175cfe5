/*
 * demap.h — C ABI of the MI355X soft-demapping library (libdemap.so, gfx950).
 *
 * The library computes, for a D-dimensional M-point constellation with a binary
 * labelling, received symbols y over AWGN with per-dimension noise variance sigma2:
 *
 *   lambda_k(y) = ln sum_{x in X_k^1} exp(-||y-x||^2/(2 sigma2))
 *               - ln sum_{x in X_k^0} exp(-||y-x||^2/(2 sigma2)),     k = 0 .. m-1,
 *
 * where X_k^b holds the points whose label has bit k equal to b, bit k being label
 * bit (m-1-k) (most significant first), and the Monte-Carlo GMI / MI estimates
 *
 *   GMI = (1/N) sum_n sum_k [1 - log2(1 + exp((1 - 2 b_{n,k}) lambda_{n,k}))]
 *   MI  = (1/N) sum_n [log2 M - log2 sum_j exp(-(||y_n-x_j||^2 - ||y_n-x_{s_n}||^2)/(2 sigma2))]
 *
 * in bits per D-dimensional symbol.  The paper's receiver takes an arbitrary,
 * non-symmetric point table and bit mapping uploaded to the GPU (Sec. 2) and its
 * geometric-shaping search scores constellations by the AWGN GMI (Sec. 5); it gives
 * no formula, so the standard bit-metric-decoding definitions above are used.
 *
 * Conventions shared by every entry point:
 *  - Every call returns a status code (DM_OK or a negative DM_E*), never throws, and
 *    stores a message retrievable with dm_last_error() on the calling thread.
 *  - Data buffers (y, tx, llr) are DEVICE pointers owned by the caller.  Small
 *    results (gmi, mi) are HOST pointers.  Constellations are uploaded from HOST
 *    arrays and owned by the library until destroyed.
 *  - All GPU work is enqueued on `stream` (a hipStream_t; NULL = the legacy default
 *    stream).  Calls that return host results synchronise that stream before
 *    returning.  Calls sharing one constellation or plan on different streams at
 *    the same time are not supported (they share library scratch).
 *  - Layouts are row-major: points M x D, y N x D (FP32), llr N x m (FP32, nats).
 *  - Limits: M = 2^m with 1 <= m <= 16, 1 <= D <= 32, 0 <= N < 2^31 per block.
 */
#ifndef DEMAP_H
#define DEMAP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    DM_OK = 0,
    DM_EINVAL = -1,       /* a null required pointer, bad size, sigma2 <= 0 or not finite,
                             labels not a bijection onto [0, M), M not a power of two */
    DM_EUNSUPPORTED = -2, /* m > 16, D > 32, or the precision is not available for this shape */
    DM_EHIP = -3,         /* a HIP runtime call failed; dm_last_error() names it */
    DM_ENOMEM = -4        /* device or host allocation failed */
};

/* Arithmetic of the distance term (the log-sum-exp always runs in FP32). */
enum {
    DM_PREC_FP32 = 0,    /* direct differences ||y-x||^2 on the vector ALU, FP32 */
    DM_PREC_BF16 = 1,    /* cross term 2y.x - ||x||^2 on MFMA, BF16 operands, FP32 accumulate */
    DM_PREC_FP16 = 2,    /* as BF16 with FP16 operands */
    DM_PREC_BF16X3 = 3,  /* BF16 hi/lo split operands, three products per term (~16-bit operands) */
    DM_PREC_FP16X3 = 4   /* FP16 hi/lo split operands, three products per term (~22-bit operands) */
};

typedef struct dm_constellation dm_constellation;

/*
 * Upload a constellation (the paper's uploaded point table + bit mapping, Sec. 2).
 *   points  HOST, M x D FP32 row-major, any row order.
 *   labels  HOST, M uint16, a bijection onto [0, M); row j carries label labels[j].
 * The library validates, reorders the table into label order, derives the MFMA
 * operand tables and uploads them to the current device.  *out is owned by the
 * caller and released with dm_constellation_destroy.
 * Errors: DM_EINVAL (null pointer, M not 2^m, labels not a bijection, non-finite
 * point), DM_EUNSUPPORTED (m > 16 or D > 32), DM_ENOMEM, DM_EHIP.
 */
int dm_constellation_create(const float* points, const uint16_t* labels, int32_t M, int32_t D,
                            dm_constellation** out);
void dm_constellation_destroy(dm_constellation* c);

/*
 * Exact bit-wise LLRs of one received block (the log-sum-exp LLRs of the header).
 *   y       DEVICE, N x D FP32.       llr  DEVICE, N x m FP32 output (nats).
 *   sigma2  noise variance per real dimension, > 0.
 *   prec    DM_PREC_*.
 * Enqueued on `stream`; does not synchronise.  N == 0 is a no-op.
 * Errors: DM_EINVAL, DM_EUNSUPPORTED, DM_EHIP, DM_ENOMEM.
 */
int dm_demap_llr(const dm_constellation* c, double sigma2, const float* y, int64_t N, float* llr,
                 int prec, void* stream);

/*
 * Monte-Carlo GMI (and MI) at n_snr noise levels over the same transmitted block
 * (the AWGN GMI the paper's shaping search evaluates, Sec. 5).
 *   sigma2  HOST, n_snr noise variances.
 *   y       HOST array of n_snr DEVICE pointers, each N x D FP32 (received block s).
 *   tx      DEVICE, N uint16 transmitted ROW indices into the uploaded point table.
 *   llr     HOST array of n_snr DEVICE pointers (N x m FP32 each) or NULL for none.
 *   gmi     HOST, n_snr FP64 outputs (bits per symbol; NaN when N == 0).
 *   mi      HOST, n_snr FP64 outputs or NULL.
 * Synchronises `stream` before returning.  The result is bit-reproducible for a
 * given input and precision (fixed-point accumulation across the grid).
 * Errors: DM_EINVAL, DM_EUNSUPPORTED, DM_EHIP, DM_ENOMEM.
 */
int dm_gmi_estimate(const dm_constellation* c, int n_snr, const double* sigma2,
                    const float* const* y, const uint16_t* tx, int64_t N, float* const* llr,
                    double* gmi, double* mi, int prec, void* stream);

/*
 * dm_gmi_estimate without any device allocation, for callers that cannot allocate: code
 * under stream capture, tight serving loops, harnesses that forbid hipMalloc.  Same
 * arguments, kernels and results (LLRs bit-identical, GMI / MI from the same fixed-point
 * sums); the launch's scratch (GMI / MI slots, fix-up counts, a fix-up queue of 2^20
 * symbols, about 16 MiB in all) is one static device array that each GPU the library runs on
 * holds until the process ends.  No hipMalloc, hipFree or allocating library call is made:
 * the constellation's MFMA operand tables are built by dm_constellation_create.
 *   Limits: n_snr <= 32 (DM_EINVAL beyond: the array holds 32 noise levels); any N < 2^31
 *   (a symbol whose part of the fix-up queue is full is recomputed in place by the demapping
 *   kernel).
 * Every call on a GPU shares that GPU's array, which keeps the last call's contents; each
 * call clears what must start at zero with a fill kernel.  Two calls whose launches overlapped
 * on one GPU would race on the array, so calls on one GPU are serialised: a host lock is held
 * from the first launch until the call has synchronised `stream` (each process has its own
 * copy of the array).
 * dm_last_fixup_count reports no counts after this call (it returns DM_EINVAL).
 * Errors: as dm_gmi_estimate; DM_EUNSUPPORTED also when an operand table is missing (after
 * the points were replaced in place).
 */
int dm_gmi_estimate_noalloc(const dm_constellation* c, int n_snr, const double* sigma2,
                            const float* const* y, const uint16_t* tx, int64_t N,
                            float* const* llr, double* gmi, double* mi, int prec, void* stream);

/*
 * Batched demapping of many instances (constellation, noise level, block) of uneven M, D and
 * N in one persistent launch (the GMI of many candidate constellations, as the paper's
 * shaping search evaluates, Sec. 5).  All instances share one operand precision `prec`.
 * Launch shape: each (M, D, prec) class runs the FP32 direct-difference body or the MFMA body
 * with work items of 1, 2 or 4 of that body's symbol tiles (1024 symbols for FP32, 512 for
 * MFMA), and workgroups claim 1, 2, 4 or 8 work items at a time.  With DM_PLAN_AUTOTUNE the
 * body and item size are chosen per class by timing every pair on a probe block that fills
 * the GPU (results cached per GPU arch in the file named by the environment variable
 * DM_AUTOTUNE_CACHE, if set) and the claim size by timing the whole plan at each; otherwise a
 * fixed rule (MFMA where it applies, one tile per item, claims of 4).  DM_PLAN_FORCE_VALU /
 * DM_PLAN_FORCE_MFMA force the body, DM_PLAN_ITEMS(k) items of 2^(k-1) tiles (k = 1..3),
 * DM_PLAN_CLAIM(k) claims of 2^(k-1) items (k = 1..4); the autotuner then picks the rest.
 * Limits: D <= 8 and M <= 4096 per instance (M <= 2048 for split MFMA operands).
 */
typedef struct dm_instance {
    const dm_constellation* c;  /* uploaded constellation (not owned) */
    double sigma2;              /* noise variance per real dimension, > 0 */
    const float* y;             /* DEVICE, N x D received symbols */
    const uint16_t* tx;         /* DEVICE, N transmitted row indices, or NULL (no GMI / MI) */
    int64_t N;
    float* llr;                 /* DEVICE, N x m LLR output (nats), or NULL */
} dm_instance;

enum { DM_PLAN_AUTOTUNE = 1, DM_PLAN_FORCE_VALU = 2, DM_PLAN_FORCE_MFMA = 4 };
#define DM_PLAN_ITEMS(k) ((int)(k) << 8)   /* force work items of 2^(k-1) symbol tiles, k = 1..3 */
#define DM_PLAN_CLAIM(k) ((int)(k) << 12)  /* force claims of 2^(k-1) work items, k = 1..4 */

typedef struct dm_plan dm_plan;

/*
 * Build a plan for n_inst instances (copied; their device buffers must stay valid for the
 * plan's lifetime): autotune if asked, list the work items (symbol tiles of each instance, the
 * most costly instance first), allocate all scratch and capture zero-fill + batched kernel +
 * fix-up into a hipGraph.  At run time each workgroup claims the next chunk of work items from
 * a device counter until the list is exhausted (dynamic balance).  Synchronous (runs timing
 * launches when autotuning).
 * Errors: DM_EINVAL, DM_EUNSUPPORTED, DM_EHIP, DM_ENOMEM.
 */
int dm_plan_create(const dm_instance* inst, int n_inst, int prec, int flags, dm_plan** out);

/* Replay the plan's graph on `stream` (asynchronous; allocates nothing). */
int dm_plan_launch(dm_plan* plan, void* stream);

/* Wait for `stream`, then return per-instance GMI and MI (HOST arrays of n_inst; NaN for
 * instances without tx or with N == 0) and fix-up pair counts (HOST int64, or NULL). */
int dm_plan_results(dm_plan* plan, double* gmi, double* mi, int64_t* fixup_pairs, void* stream);

/* Per-instance launch shape (any output may be NULL): kernel body (0 = FP32, 1 = MFMA), its
 * cost in ns per (symbol, point) and the symbols per work item. */
int dm_plan_info(const dm_plan* plan, int* kinds, double* ns_per_pair, int32_t* item_symbols);

/* Launch shape of a plan (any output may be NULL): work items in its list, items a workgroup
 * claims at a time, and workgroups of the persistent launch. */
int dm_plan_stats(const dm_plan* plan, int64_t* n_items, int32_t* claim_items, int32_t* grid);

void dm_plan_destroy(dm_plan* plan);

/* One-shot: create, launch, read results, destroy (synchronous). */
int dm_demap_batched(const dm_instance* inst, int n_inst, int prec, int flags, double* gmi, double* mi,
                     void* stream);

/*
 * Exact LLRs with one noise variance per symbol (the learned demapper's training targets are
 * drawn at continuously distributed SNRs; also usable for fading channels).
 *   sigma2  DEVICE, N FP32 per-symbol variances.  Entries that are not finite and > 0 give
 *           non-finite LLRs for their symbols (never a fault).
 *   prec    DM_PREC_FP32, DM_PREC_BF16 or DM_PREC_BF16X3 (the FP16 operand range depends on
 *           1/sigma2, which the host cannot bound without reading the array).
 * Enqueued on `stream`; does not synchronise.  Errors: as dm_demap_llr.
 */
int dm_demap_llr_var(const dm_constellation* c, const float* sigma2, const float* y, int64_t N, float* llr,
                     int prec, void* stream);

/* ------------------------------------------------------------------------------------------
 * Learned demapper.  This is a project addition with no passage in the paper: the paper's
 * receiver demaps by minimum distance (Sec. 2) and mentions no learned demapping.  The network
 * judged by the exact path of this library (its fallback and its GMI-loss audit) is an
 * MLP (D+1) -> 256 -> 256 -> m with tanh-form GELU, BF16 weights and activations and FP32
 * accumulation in training, whose m outputs estimate the exact LLRs (nats).  Inference keeps
 * the first layer in BF16 and evaluates the GELU in packed FP16 (within 1.2e-3 of the tanh
 * form's Phi in x Phi(x), dm_probe_gelu) feeding FP16 operands to layers 2 and 3, the hidden
 * layers on a quarter scale; hidden pre-activations beyond +-262016 saturate and |W3| should
 * stay below 16376.  Its inputs are y and the SNR
 * feature (s - 7.5) / 7.5 with s = -10 log10(2 sigma2), the SNR in dB of a constellation with
 * unit energy per two real dimensions.  Training minimises the soft binary cross-entropy
 * between sigmoid(output) and sigmoid(exact LLR), averaged over samples and bits, with Adam on
 * FP32 master weights.  A network is bound to the constellation it was created for.
 *
 * Weight arrays (HOST, FP32, dm_mlp_param_count(D, m) values) are ordered
 *   W1 [(D+1) x 256] row-major (out = x W + b), b1 [256], W2 [256 x 256], b2 [256],
 *   W3 [256 x m], b3 [m].
 * ---------------------------------------------------------------------------------------- */
typedef struct dm_mlp dm_mlp;

/* (D+1)*256 + 256 + 256*256 + 256 + 256*m + m, or DM_EINVAL unless 1 <= D <= 13 and 1 <= m <= 32. */
int64_t dm_mlp_param_count(int32_t D, int32_t m);

/*
 * Create a network for constellation c with the given initial weights (HOST, copied).  Its
 * trained SNR range starts unbounded; dm_mlp_train sets it.
 * Errors: DM_EINVAL (null, non-finite weight), DM_EUNSUPPORTED (D > 13 or m > 32), DM_ENOMEM, DM_EHIP.
 */
int dm_mlp_create(const dm_constellation* c, const float* weights, dm_mlp** out);
void dm_mlp_destroy(dm_mlp* net);
/* FP32 master weights to HOST `weights` (synchronises the device). */
int dm_mlp_get_weights(const dm_mlp* net, float* weights);
/* Replace the weights (HOST) and reset the Adam state (synchronises the device). */
int dm_mlp_set_weights(dm_mlp* net, const float* weights);
/* Adam steps taken and the trained SNR range in dB (any output may be NULL). */
int dm_mlp_info(const dm_mlp* net, int64_t* steps, double* snr_lo_db, double* snr_hi_db);

typedef struct dm_train_config {
    int32_t batch;             /* samples per Adam step: a multiple of 256 in [256, 65536] */
    int32_t epochs;            /* passes over the samples, >= 1 */
    float lr, lr_final;        /* cosine decay from lr (first step) to lr_final (last step) */
    float beta1, beta2, eps;   /* Adam; a value <= 0 selects 0.9, 0.999, 1e-8 */
    int32_t target_prec;       /* exact-target precision: DM_PREC_FP32, DM_PREC_BF16 or DM_PREC_BF16X3 */
    double snr_lo_db, snr_hi_db;  /* SNR range (s above) the samples cover; becomes the trained range */
} dm_train_config;

/*
 * Train on N samples.  y DEVICE N x D received symbols, sigma2 DEVICE N FP32 noise variance of
 * each sample.  The exact LLRs of each sample under its own sigma2 (computed with c, chunk by
 * chunk) are the targets; batches are taken in order; the last N % batch samples of each epoch
 * are not used.  loss (HOST, may be NULL): mean loss over the last min(64, steps) steps.
 * Synchronises `stream`.  Errors: DM_EINVAL (bad config, N < batch, another constellation),
 * DM_EUNSUPPORTED, DM_ENOMEM, DM_EHIP.
 */
int dm_mlp_train(dm_mlp* net, const dm_constellation* c, const dm_train_config* cfg, const float* y,
                 const float* sigma2, int64_t N, double* loss, void* stream);

/*
 * Loss gradients at the current weights for one batch of B samples (a multiple of 256) with
 * given targets, without updating anything: y DEVICE B x D, sigma2 DEVICE B FP32, target
 * DEVICE B x m FP32 (nats).  grads HOST (weight order above), loss HOST or NULL.
 * Synchronises `stream`.
 */
int dm_mlp_gradients(dm_mlp* net, const float* y, const float* sigma2, const float* target, int32_t B,
                     float* grads, double* loss, void* stream);

typedef struct dm_learned_opts {
    double max_gmi_loss;  /* bits per symbol; an audited point whose estimated GMI loss exceeds
                             this is recomputed exactly.  < 0 disables the audit. */
    int32_t audit_log2;   /* the audit covers the first max(ceil(N / 2^audit_log2), 8192) symbols */
    int32_t exact_prec;   /* DM_PREC_* of the audit and of every exact fallback */
} dm_learned_opts;  /* NULL selects {0.01, 6, DM_PREC_FP32} */

enum {
    DM_LEARNED_OK = 0,             /* the network's LLRs and GMI are returned */
    DM_FALLBACK_AUDIT = 1,         /* audit loss above the bound: exact results returned */
    DM_FALLBACK_SNR = 2,           /* SNR outside the trained range: exact results returned */
    DM_FALLBACK_CONSTELLATION = 3  /* c is not the network's constellation: exact results returned */
};

/*
 * Learned demapping of one transmitted block at n_snr noise levels (same arguments as
 * dm_gmi_estimate, tx and llr optional).  Per point: if the network covers it, its LLRs are
 * written and, with tx, its GMI is estimated; the audit then runs the exact path on the
 * block's prefix and estimates the GMI loss as exact minus learned GMI over that prefix.  Points
 * that fail a check are recomputed exactly over the whole block (LLRs overwritten).
 *   gmi            HOST n_snr (required with tx; NaN for N == 0).
 *   gmi_loss       HOST n_snr or NULL: the audit's loss estimate (NaN when not audited).
 *   used_fallback  HOST n_snr: DM_LEARNED_OK or the DM_FALLBACK_* reason.
 * Synchronises `stream`.  Errors: as dm_gmi_estimate.
 */
int dm_demap_learned(dm_mlp* net, const dm_constellation* c, int n_snr, const double* sigma2,
                     const float* const* y, const uint16_t* tx, int64_t N, float* const* llr,
                     const dm_learned_opts* opts, double* gmi, double* gmi_loss, int* used_fallback,
                     void* stream);

/* Checkpoint: weights, Adam state, step count, trained SNR range and constellation identity in
 * a little-endian binary file with a versioned header. */
int dm_mlp_save(const dm_mlp* net, const char* path);
/* Load a checkpoint for constellation c (same D and m required; the recorded identity is kept,
 * so a different table makes dm_demap_learned fall back). */
int dm_mlp_load(const dm_constellation* c, const char* path, dm_mlp** out);

/*
 * Hard decisions: the minimum-Euclidean-distance point of each received symbol (the
 * paper's receiver decides symbols by minimum distance over the uploaded table, Sec. 2) and,
 * with tx, the symbol- and bit-error counts behind its BER / Q-factor figures (Sec. 4).
 *   y           HOST array of n_blk DEVICE pointers, each N x D FP32.
 *   tx          DEVICE, N uint16 transmitted ROW indices; required when counting, else may be NULL.
 *   labels_out  HOST array of n_blk DEVICE pointers (N uint16 decided LABELS each) or NULL.
 *   sym_err, bit_err  HOST int64 n_blk outputs, or NULL (no counting).
 *   method      DM_HARD_AUTO, DM_HARD_VALU or DM_HARD_MFMA (see below); all give the same decisions.
 *   n_exact     HOST int64 or NULL: symbols the MFMA method passed to the exact path.
 * The decision is defined by FP32 distances t_d = y_d - x_d, acc = fma(t_d, t_d, acc) for
 * d = 0..D-1 from acc = 0, ties to the lowest label.  DM_HARD_VALU evaluates exactly that for
 * every point.  DM_HARD_MFMA (M >= 32, D <= 8, point norms^2 < 60000) ranks the points with a
 * split-FP16 MFMA cross term and accepts its winner only when the gap to the runner-up exceeds
 * twice a bound on the error of both computations; other symbols are decided by the FP32
 * formula.  DM_HARD_AUTO picks DM_HARD_MFMA when it applies.  Bit errors are the popcount of
 * (decided label XOR sent label).  Synchronises `stream` when counting or when n_exact is given.
 * Errors: DM_EINVAL, DM_EUNSUPPORTED, DM_EHIP, DM_ENOMEM.
 */
enum { DM_HARD_AUTO = 0, DM_HARD_VALU = 1, DM_HARD_MFMA = 2 };
int dm_hard_decision(const dm_constellation* c, int n_blk, const float* const* y, const uint16_t* tx, int64_t N,
                     uint16_t* const* labels_out, int64_t* sym_err, int64_t* bit_err, int32_t method,
                     int64_t* n_exact, void* stream);

/* Q-factor in dB from a bit-error ratio, 20 log10(sqrt(2) erfcinv(2 BER)) (the usual Gaussian
 * reading; the paper quotes Q-factors without a formula).  NaN unless 0 < ber < 0.5. */
double dm_q_factor_db(double ber);

/*
 * Geometric-shaping search by AWGN GMI (the paper's iterative design of its GS constellations,
 * Sec. 5): from the given constellation, each iteration proposes `candidates` modifications of
 * the current one -- with probability swap_prob the labels of two random points are swapped,
 * otherwise one random point moves by perturb_sd * N(0, I) and the constellation is rescaled to
 * unit energy per two dimensions -- evaluates all of them in one batched FP32 GMI launch on the
 * common block (tx, z) at snr_db, and keeps the best one if its GMI exceeds the current GMI.
 * Random draws come from SplitMix64 seeded with `seed`.
 *   points, labels  HOST initial constellation (M x D, any row order; rescaled to unit energy).
 *   tx              DEVICE, N uint16 transmitted LABELS.   z  DEVICE, N x D FP32 unit noise.
 *   out_points      HOST M x D result in label order (row l carries label l).
 *   gmi_trace       HOST iters + 1 values: the current GMI after each iteration (index 0: start).
 *   accepted        HOST, number of accepted iterations, or NULL.
 * Limits: M a power of two <= 4096, D <= 8, 1 <= candidates <= 64.  Device memory: candidates
 * x N x D FP32 received blocks.  Synchronous.  Errors: DM_EINVAL, DM_EUNSUPPORTED, DM_ENOMEM, DM_EHIP.
 */
typedef struct dm_gs_config {
    double snr_db;       /* SNR (unit energy per 2D) of the AWGN GMI */
    int32_t iters;       /* iterations, >= 0 */
    int32_t candidates;  /* modifications evaluated per iteration, 1..64 */
    double perturb_sd;   /* standard deviation of a point move (per dimension) */
    double swap_prob;    /* probability that a modification is a label swap */
    uint64_t seed;
} dm_gs_config;

int dm_gs_optimize(const float* points, const uint16_t* labels, int32_t M, int32_t D, const dm_gs_config* cfg,
                   const uint16_t* tx, const float* z, int64_t N, float* out_points, double* gmi_trace,
                   int32_t* accepted, void* stream);

/*
 * Streamed demapping of host-resident data (the paper's receiver handles fixed-size sample
 * buffers as they arrive, Sec. 2): the host block is processed in buffers of buffer_symbols
 * symbols cycling through n_buffers slots of pinned staging and device memory; each buffer's
 * host-to-device copy, demapping and device-to-host copy run on three streams of default
 * priority, so transfers of one buffer overlap the demapping of another.
 * dm_streamer_run: y HOST N x D FP32 (any host memory; page-locked memory is transferred
 * directly, other memory through the pinned staging), llr HOST N x m FP32 output (nats),
 * seconds HOST wall time of the call or NULL.  Synchronous: returns when every LLR is in llr.
 * LLRs are identical to dm_demap_llr on the whole block.  Limits: 1 <= buffer_symbols <= 2^26,
 * 2 <= n_buffers <= 16.  Errors: DM_EINVAL, DM_EUNSUPPORTED, DM_ENOMEM, DM_EHIP.
 */
typedef struct dm_streamer dm_streamer;
int dm_streamer_create(const dm_constellation* c, int64_t buffer_symbols, int32_t n_buffers, int32_t prec,
                       dm_streamer** out);
int dm_streamer_run(dm_streamer* s, double sigma2, const float* y, int64_t N, float* llr, double* seconds);
void dm_streamer_destroy(dm_streamer* s);

/* Number of (symbol, bit) pairs that the last call on this thread sent through the
 * far-subset underflow fix-up, per SNR point (HOST array of n_snr, may be NULL).
 * Returns the total, or a negative DM_E* if no call has run on this thread. */
int64_t dm_last_fixup_count(int64_t* per_snr, int n_snr);

/* Thread-local description of the last error on the calling thread ("" if none). */
const char* dm_last_error(void);

/* Library version string. */
const char* dm_version(void);

#ifdef __cplusplus
}
#endif

#endif /* DEMAP_H */
