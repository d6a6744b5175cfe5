/*
 * FP64 CPU oracle for exact soft demapping and Monte-Carlo GMI / MI.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU-baseline
 * leg of the benchmark may load this file's library.  It shares no code, header,
 * table or constant with the GPU library and must never be linked into it.
 *
 * What it computes (the paper uses "the GMI for the AWGN channel" as the figure of
 * merit of its geometric-shaping search (Sec. 5, Discussion) and uploads an arbitrary
 * point table plus bit mapping to its receiver (Sec. 2) but prints no formula; the
 * definitions below are the standard bit-metric-decoding ones, one reading each):
 *
 *   AWGN per real dimension with variance sigma2:  p(y|x) ~ exp(-||y-x||^2 / (2 sigma2)).
 *   Bit k of a label (k = 0 .. m-1) is label bit (m-1-k): most significant first.
 *   X_k^b = { x_j : bit k of labels[j] equals b }.
 *   LLR  lambda_k = ln sum_{X_k^1} exp(-d_j/(2 sigma2)) - ln sum_{X_k^0} exp(-d_j/(2 sigma2)),
 *        d_j = ||y - x_j||^2, each log-sum-exp taken with its own subset maximum.
 *   Per-symbol GMI term  g_n = sum_k [ 1 - log2(1 + exp((1 - 2 b_{n,k}) lambda_k)) ],
 *        b_{n,k} = bit k of the transmitted label.
 *   Per-symbol MI term   i_n = log2 M - log2 sum_j exp(-(d_j - d_tx)/(2 sigma2)).
 *   GMI = (1/N) sum_n g_n,  MI = (1/N) sum_n i_n   (Neumaier-compensated FP64 sums).
 *
 * Inputs are the same FP32 arrays the GPU receives, promoted exactly to FP64.
 * All arithmetic is FP64 with libm exp/log/log1p; no blocking, no fusion.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_OK 0
#define ORACLE_EINVAL (-1)

static int ilog2_exact(int M) {
    int m = 0;
    while ((1 << m) < M) m++;
    return ((1 << m) == M) ? m : -1;
}

static int label_bit(unsigned label, int m, int k) { return (int)((label >> (m - 1 - k)) & 1u); }

/* log(1 + exp(z)) without overflow. */
static double softplus(double z) { return (z > 0.0 ? z : 0.0) + log1p(exp(-fabs(z))); }

/* Neumaier compensated accumulation. */
typedef struct { double s, c; } nsum;
static void nsum_add(nsum* a, double v) {
    double t = a->s + v;
    if (fabs(a->s) >= fabs(v)) a->c += (a->s - t) + v;
    else a->c += (v - t) + a->s;
    a->s = t;
}
static double nsum_get(const nsum* a) { return a->s + a->c; }

/*
 * Log-sum-exp of v[j] = -d[j]/(2 sigma2) over the points whose label has bit k equal
 * to b (k < 0 selects every point).  Two passes: the subset maximum, then the sum of
 * exp(v - max).  Returns -INFINITY for an empty subset.
 */
static double subset_lse(const double* v, const uint16_t* labels, int M, int m, int k, int b) {
    double mx = -INFINITY;
    for (int j = 0; j < M; j++) {
        if (k >= 0 && label_bit(labels[j], m, k) != b) continue;
        if (v[j] > mx) mx = v[j];
    }
    if (mx == -INFINITY) return -INFINITY;
    double s = 0.0;
    for (int j = 0; j < M; j++) {
        if (k >= 0 && label_bit(labels[j], m, k) != b) continue;
        s += exp(v[j] - mx);
    }
    return mx + log(s);
}

/*
 * Exact per-symbol LLRs, GMI terms and MI terms.
 *   points  M x D row-major FP32 (any row order), labels M (a bijection onto [0, M)).
 *   y       N x D row-major FP32 received symbols, tx N transmitted row indices.
 *   llr     N x m FP64 output or NULL; g, mi: N FP64 outputs or NULL.
 *   gmi, mi_mean: FP64 means over the N symbols (NaN when N == 0), may be NULL.
 *   nthreads <= 0 uses the OpenMP default.
 * Returns ORACLE_OK or ORACLE_EINVAL (bad sizes, sigma2 <= 0, labels not a bijection).
 */
int oracle_demap(int M, int D, const float* points, const uint16_t* labels, double sigma2,
                 const float* y, const uint16_t* tx, int64_t N, double* llr, double* g, double* mi,
                 double* gmi, double* mi_mean, int nthreads) {
    int m = ilog2_exact(M);
    if (m < 1 || m > 16 || D < 1 || N < 0 || !(sigma2 > 0.0) || !isfinite(sigma2)) return ORACLE_EINVAL;
    if (!points || !labels || (N > 0 && (!y || !tx))) return ORACLE_EINVAL;
    {
        unsigned char* seen = (unsigned char*)calloc((size_t)M, 1);
        if (!seen) return ORACLE_EINVAL;
        for (int j = 0; j < M; j++) {
            if (labels[j] >= M || seen[labels[j]]) { free(seen); return ORACLE_EINVAL; }
            seen[labels[j]] = 1;
        }
        free(seen);
    }
    for (int64_t n = 0; n < N; n++)
        if (tx[n] >= M) return ORACLE_EINVAL;

    nsum gs = {0.0, 0.0}, ms = {0.0, 0.0};
    double* gbuf = (double*)malloc(sizeof(double) * (size_t)(N > 0 ? N : 1));
    double* mbuf = (double*)malloc(sizeof(double) * (size_t)(N > 0 ? N : 1));
    if (!gbuf || !mbuf) { free(gbuf); free(mbuf); return ORACLE_EINVAL; }
    const double two_s2 = 2.0 * sigma2;

#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel
#endif
    {
        double* v = (double*)malloc(sizeof(double) * (size_t)M);
#ifdef _OPENMP
#pragma omp for schedule(static)
#endif
        for (int64_t n = 0; n < N; n++) {
            /* v_j = -||y - x_j||^2 / (2 sigma2) */
            for (int j = 0; j < M; j++) {
                double d = 0.0;
                for (int e = 0; e < D; e++) {
                    double diff = (double)y[n * D + e] - (double)points[(int64_t)j * D + e];
                    d += diff * diff;
                }
                v[j] = -d / two_s2;
            }
            unsigned txl = labels[tx[n]];
            double gn = 0.0;
            for (int k = 0; k < m; k++) {
                double lam = subset_lse(v, labels, M, m, k, 1) - subset_lse(v, labels, M, m, k, 0);
                if (llr) llr[n * m + k] = lam;
                int b = label_bit(txl, m, k);
                double s = (b == 0) ? lam : -lam; /* (1 - 2b) * lambda */
                gn += 1.0 - softplus(s) / log(2.0);
            }
            /* i_n = log2 M - log2 sum_j exp(v_j - v_tx) */
            double lse_all = subset_lse(v, labels, M, m, -1, 0);
            double in = (double)m - (lse_all - v[tx[n]]) / log(2.0);
            gbuf[n] = gn;
            mbuf[n] = in;
            if (g) g[n] = gn;
            if (mi) mi[n] = in;
        }
        free(v);
    }
    /* Sequential compensated means, in symbol order, independent of the thread count. */
    for (int64_t n = 0; n < N; n++) { nsum_add(&gs, gbuf[n]); nsum_add(&ms, mbuf[n]); }
    free(gbuf);
    free(mbuf);
    if (gmi) *gmi = (N > 0) ? nsum_get(&gs) / (double)N : NAN;
    if (mi_mean) *mi_mean = (N > 0) ? nsum_get(&ms) / (double)N : NAN;
    return ORACLE_OK;
}

/* GMI from given LLRs (nats) and transmitted labels: the same per-bit term as above. */
int oracle_gmi_from_llr(int m, const double* llr, const uint16_t* tx_label, int64_t N, double* gmi) {
    if (m < 1 || m > 16 || N < 0 || !gmi) return ORACLE_EINVAL;
    nsum gs = {0.0, 0.0};
    for (int64_t n = 0; n < N; n++) {
        double gn = 0.0;
        for (int k = 0; k < m; k++) {
            int b = label_bit(tx_label[n], m, k);
            double lam = llr[n * m + k];
            double s = (b == 0) ? lam : -lam;
            gn += 1.0 - softplus(s) / log(2.0);
        }
        nsum_add(&gs, gn);
    }
    *gmi = (N > 0) ? nsum_get(&gs) / (double)N : NAN;
    return ORACLE_OK;
}

int oracle_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/*
 * Hard decisions by minimum Euclidean distance (the receiver's decision rule, Sec. 2) and
 * their symbol / bit errors against the transmitted labels (the BER behind the paper's
 * Q-factors, Sec. 4).  The decision is an integer taken from floating-point distances, so it
 * is taken in the single-precision formula the library documents: t_d = y_d - x_d,
 * acc = fmaf(t_d, t_d, acc) over d = 0..D-1 starting from 0.  Every row is scanned; the
 * smallest distance wins and equal distances go to the smallest label.  A NaN distance never
 * wins.  out_label (N) may be NULL; tx (N rows) may be NULL, then the counts are not formed.
 */
int oracle_hard_demap(int M, int D, const float* points, const uint16_t* labels, const float* y,
                      const uint16_t* tx, int64_t N, uint16_t* out_label, int64_t* sym_err, int64_t* bit_err) {
    if (M < 1 || D < 1 || N < 0 || !points || !labels || (N > 0 && !y)) return ORACLE_EINVAL;
    int64_t se = 0, be = 0;
    for (int64_t n = 0; n < N; ++n) {
        float best = INFINITY;
        int best_label = -1;
        for (int j = 0; j < M; ++j) {
            float acc = 0.0f;
            for (int d = 0; d < D; ++d) {
                const float t = y[n * D + d] - points[(size_t)j * D + d];
                acc = fmaf(t, t, acc);
            }
            if (acc < best || (acc == best && labels[j] < best_label)) {
                best = acc;
                best_label = labels[j];
            }
        }
        if (best_label < 0) { /* every distance NaN: the lowest label */
            best_label = M;
            for (int j = 0; j < M; ++j)
                if (labels[j] < best_label) best_label = labels[j];
        }
        if (out_label) out_label[n] = (uint16_t)best_label;
        if (tx) {
            if (tx[n] >= M) return ORACLE_EINVAL;
            const unsigned diff = (unsigned)best_label ^ labels[tx[n]];
            se += diff != 0;
            for (unsigned v = diff; v; v >>= 1) be += v & 1u;
        }
    }
    if (sym_err) *sym_err = se;
    if (bit_err) *bit_err = be;
    return ORACLE_OK;
}
