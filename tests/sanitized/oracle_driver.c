/*
 * Driver that runs the FP64 oracle under AddressSanitizer and UndefinedBehaviorSanitizer
 * (test infrastructure: built and run by tests/test_oracle_sanitized.py, never by the library).
 *
 * It calls every exported oracle function on closed-form cases, edge cases (N = 0 and 1, M = 2,
 * D = 1, permuted labels, a 4096-point table, NaN inputs, ties) and invalid arguments, so that
 * any out-of-bounds access, use of uninitialised memory or undefined arithmetic on those paths
 * aborts the run; it also checks the closed forms themselves.  Exit status: number of failures.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int oracle_demap(int M, int D, const float* points, const uint16_t* labels, double sigma2, const float* y,
                 const uint16_t* tx, int64_t N, double* llr, double* g, double* mi, double* gmi, double* mi_mean,
                 int nthreads);
int oracle_gmi_from_llr(int m, const double* llr, const uint16_t* tx_label, int64_t N, double* gmi);
int oracle_hard_demap(int M, int D, const float* points, const uint16_t* labels, const float* y, const uint16_t* tx,
                      int64_t N, uint16_t* out_label, int64_t* sym_err, int64_t* bit_err);
int oracle_max_threads(void);

static int failures = 0;
#define CHECK(cond, ...)                   \
    do {                                   \
        if (!(cond)) {                     \
            ++failures;                    \
            printf("FAIL: " __VA_ARGS__); \
            printf("\n");                  \
        }                                  \
    } while (0)

static uint64_t rng_state = 0x9E3779B97F4A7C15ull;
static double urand(void) { /* SplitMix64 -> [0, 1) */
    uint64_t z = (rng_state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (double)(z >> 11) * 0x1.0p-53;
}
static double nrand(void) { return sqrt(-2.0 * log(1.0 - urand())) * cos(6.283185307179586 * urand()); }

/* DP-QPSK: per dimension +-A with label bit (m-1-d) = (x_d > 0): lambda_d = 2 A y_d / sigma2. */
static void qpsk_closed_form(void) {
    enum { M = 16, D = 4, N = 257 };
    float pts[M * D];
    uint16_t lab[M];
    const float A = (float)(1.0 / sqrt(2.0));
    for (int j = 0; j < M; ++j) {
        lab[j] = (uint16_t)(M - 1 - j); /* a row order that is not label order */
        for (int d = 0; d < D; ++d) pts[j * D + d] = ((lab[j] >> (D - 1 - d)) & 1) ? A : -A;
    }
    float y[N * D];
    uint16_t tx[N];
    for (int n = 0; n < N; ++n) {
        tx[n] = (uint16_t)(urand() * M);
        for (int d = 0; d < D; ++d) y[n * D + d] = (float)(pts[tx[n] * D + d] + 0.6 * nrand());
    }
    double llr[N * D], g[N], mi[N], gmi, mim;
    const double s2 = 0.3;
    int rc = oracle_demap(M, D, pts, lab, s2, y, tx, N, llr, g, mi, &gmi, &mim, 0);
    CHECK(rc == 0, "qpsk rc %d", rc);
    double worst = 0.0;
    for (int n = 0; n < N; ++n)
        for (int k = 0; k < D; ++k) {
            const double want = 2.0 * (double)A * (double)y[n * D + k] / s2;
            const double e = fabs(llr[n * D + k] - want) / fmax(1.0, fabs(want));
            if (e > worst) worst = e;
        }
    CHECK(worst <= 1e-12, "qpsk closed-form LLR error %g", worst);
    CHECK(gmi <= mim + 1e-12 && mim <= 4.0 && gmi > 0.0, "qpsk gmi %g mi %g", gmi, mim);
    double g2;
    uint16_t tl[N];
    for (int n = 0; n < N; ++n) tl[n] = lab[tx[n]];
    rc = oracle_gmi_from_llr(D, llr, tl, N, &g2);
    CHECK(rc == 0 && fabs(g2 - gmi) <= 1e-12, "gmi_from_llr %g vs %g", g2, gmi);
}

/* M = 2: lambda = (||y - x0||^2 - ||y - x1||^2) / (2 sigma2), x1 the point labelled 1. */
static void two_points(int D) {
    float pts[2 * 8];
    uint16_t lab[2] = {1, 0};
    for (int i = 0; i < 2 * D; ++i) pts[i] = (float)nrand();
    enum { N = 33 };
    float y[N * 8];
    uint16_t tx[N];
    for (int n = 0; n < N; ++n) {
        tx[n] = (uint16_t)(n & 1);
        for (int d = 0; d < D; ++d) y[n * D + d] = (float)nrand();
    }
    double llr[N];
    int rc = oracle_demap(2, D, pts, lab, 0.7, y, tx, N, llr, NULL, NULL, NULL, NULL, 1);
    CHECK(rc == 0, "M=2 rc %d", rc);
    for (int n = 0; n < N; ++n) {
        double d0 = 0, d1 = 0;
        for (int d = 0; d < D; ++d) {
            const double a = (double)y[n * D + d] - pts[1 * D + d]; /* row 1 has label 0 */
            const double b = (double)y[n * D + d] - pts[0 * D + d]; /* row 0 has label 1 */
            d0 += a * a;
            d1 += b * b;
        }
        const double want = (d0 - d1) / 1.4;
        CHECK(fabs(llr[n] - want) <= 1e-12 * fmax(1.0, fabs(want)), "M=2 D=%d n=%d %g vs %g", D, n, llr[n], want);
    }
}

static void edge_cases(void) {
    /* N = 0: NaN means, no access to y or tx */
    float p2[2] = {-1.0f, 1.0f};
    uint16_t l2[2] = {0, 1};
    double gmi = 0, mim = 0;
    int rc = oracle_demap(2, 1, p2, l2, 1.0, NULL, NULL, 0, NULL, NULL, NULL, &gmi, &mim, 0);
    CHECK(rc == 0 && isnan(gmi) && isnan(mim), "N=0 rc %d gmi %g", rc, gmi);
    rc = oracle_gmi_from_llr(3, NULL, NULL, 0, &gmi);
    CHECK(rc == 0 && isnan(gmi), "gmi_from_llr N=0");
    /* N = 1, D = 1 */
    float y1 = 0.25f;
    uint16_t t1 = 1;
    double l1, g1, m1;
    rc = oracle_demap(2, 1, p2, l2, 0.5, &y1, &t1, 1, &l1, &g1, &m1, &gmi, &mim, 0);
    CHECK(rc == 0 && fabs(l1 - 2.0 * 0.25 / 0.5) <= 1e-15, "N=1 llr %g", l1);
    /* a 4096-point, 3-D table with permuted labels and a ragged block */
    enum { M = 4096, D = 3, N = 37 };
    float* pts = (float*)malloc(sizeof(float) * M * D);
    uint16_t* lab = (uint16_t*)malloc(sizeof(uint16_t) * M);
    for (int j = 0; j < M; ++j) lab[j] = (uint16_t)j;
    for (int j = M - 1; j > 0; --j) { /* Fisher-Yates */
        const int k = (int)(urand() * (j + 1));
        const uint16_t t = lab[j];
        lab[j] = lab[k];
        lab[k] = t;
    }
    for (int i = 0; i < M * D; ++i) pts[i] = (float)nrand();
    float y[N * D];
    uint16_t tx[N];
    for (int n = 0; n < N; ++n) {
        tx[n] = (uint16_t)(urand() * M);
        for (int d = 0; d < D; ++d) y[n * D + d] = pts[tx[n] * D + d] + (float)(0.05 * nrand());
    }
    double* llr = (double*)malloc(sizeof(double) * N * 12);
    double g[N], mi[N];
    rc = oracle_demap(M, D, pts, lab, 0.01, y, tx, N, llr, g, mi, &gmi, &mim, 0);
    CHECK(rc == 0 && isfinite(gmi) && isfinite(mim) && mim <= 12.0 + 1e-12, "M=4096 rc %d gmi %g mi %g", rc, gmi, mim);
    for (int n = 0; n < N; ++n) CHECK(g[n] <= 12.0 + 1e-12 && mi[n] <= 12.0 + 1e-12, "per-symbol terms above m");
    /* invalid arguments: labels not a bijection, M not a power of two, tx >= M, sigma2 <= 0 */
    uint16_t bad[4] = {0, 1, 1, 3};
    float p4[4] = {0, 1, 2, 3};
    float yy[1] = {0.5f};
    uint16_t tt[1] = {0};
    CHECK(oracle_demap(4, 1, p4, bad, 1.0, yy, tt, 1, NULL, NULL, NULL, NULL, NULL, 0) != 0, "duplicate label accepted");
    CHECK(oracle_demap(3, 1, p4, l2, 1.0, yy, tt, 1, NULL, NULL, NULL, NULL, NULL, 0) != 0, "M=3 accepted");
    uint16_t big[1] = {9};
    uint16_t l4[4] = {0, 1, 2, 3};
    CHECK(oracle_demap(4, 1, p4, l4, 1.0, yy, big, 1, NULL, NULL, NULL, NULL, NULL, 0) != 0, "tx >= M accepted");
    CHECK(oracle_demap(4, 1, p4, l4, 0.0, yy, tt, 1, NULL, NULL, NULL, NULL, NULL, 0) != 0, "sigma2 = 0 accepted");
    CHECK(oracle_demap(4, 1, p4, l4, NAN, yy, tt, 1, NULL, NULL, NULL, NULL, NULL, 0) != 0, "sigma2 NaN accepted");
    /* hard decisions: ties go to the lowest label (y = 1: labels 2 and 1; y = 0: labels 3, 2, 1),
       a NaN symbol gets the lowest label */
    float ph[4] = {-1.0f, 1.0f, 1.0f, 3.0f};
    uint16_t lh[4] = {3, 2, 1, 0};
    float yh[3] = {1.0f, NAN, 0.0f};
    uint16_t th[3] = {2, 0, 0};
    uint16_t out[3];
    int64_t se = -1, be = -1;
    rc = oracle_hard_demap(4, 1, ph, lh, yh, th, 3, out, &se, &be);
    CHECK(rc == 0 && out[0] == 1 && out[1] == 0 && out[2] == 1, "hard decisions %u %u %u", out[0], out[1], out[2]);
    CHECK(se == 2 && be == 3, "hard decision errors %lld %lld", (long long)se, (long long)be);
    free(pts);
    free(lab);
    free(llr);
}

int main(void) {
    qpsk_closed_form();
    for (int D = 1; D <= 8; ++D) two_points(D);
    edge_cases();
    printf("oracle under sanitizers: %d failure(s), %d OpenMP threads\n", failures, oracle_max_threads());
    return failures;
}
