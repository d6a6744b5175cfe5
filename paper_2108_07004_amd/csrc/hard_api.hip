// C ABI of hard-decision (minimum-distance) demapping, error counting and the Q-factor.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>
#include <mutex>

#include "api_internal.hpp"
#include "kernels.hpp"

using dmapi::fail;

extern "C" {

int dm_hard_decision(const dm_constellation* cc, int n_blk, const float* const* y, const uint16_t* tx, int64_t N,
                     uint16_t* const* labels_out, int64_t* sym_err, int64_t* bit_err, int32_t method,
                     int64_t* n_exact, void* stream) {
    dmapi::clear_error();
    auto* c = const_cast<dm_constellation*>(cc);
    if (!c || !y) return fail(DM_EINVAL, "null argument");
    if (n_blk < 1) return fail(DM_EINVAL, "n_blk=%d < 1", n_blk);
    if (N < 0 || N >= (int64_t(1) << 31)) return fail(DM_EINVAL, "N=%lld out of range", (long long)N);
    if (method < DM_HARD_AUTO || method > DM_HARD_MFMA) return fail(DM_EINVAL, "unknown method %d", method);
    const bool counting = sym_err || bit_err;
    if (n_exact) *n_exact = 0;
    if (N == 0) {  // no symbols: nothing to read (empty device buffers may be null)
        for (int s = 0; s < n_blk; ++s) {
            if (sym_err) sym_err[s] = 0;
            if (bit_err) bit_err[s] = 0;
        }
        return DM_OK;
    }
    const bool mfma_ok = c->M >= 32 && c->D <= 8 && c->max_norm < 60000.0f;
    if (method == DM_HARD_MFMA && !mfma_ok)
        return fail(DM_EUNSUPPORTED, "MFMA decisions need M >= 32, D <= 8 and point norms inside the FP16 range");
    const bool use_mfma = method == DM_HARD_MFMA || (method == DM_HARD_AUTO && mfma_ok);
    if (counting && !tx) return fail(DM_EINVAL, "error counts need the transmitted rows (tx)");
    int r;
    if ((r = dmapi::check_current_device(c))) return r;
    if (counting && (r = dmapi::check_device_ptr(tx, "tx", c->device))) return r;
    for (int s = 0; s < n_blk; ++s) {
        if ((r = dmapi::check_device_ptr(y[s], "y[s]", c->device))) return r;
        if (labels_out && (r = dmapi::check_device_ptr(labels_out[s], "labels_out[s]", c->device))) return r;
    }
    std::lock_guard<std::mutex> lock(c->mu);
    if ((r = dmapi::ensure_scratch(c, use_mfma ? (uint64_t)N * std::min(n_blk, dm::kMaxSnrPerLaunch) : 0))) return r;
    if (use_mfma && (r = dmapi::ensure_frag(c, DM_PREC_FP16X3, false))) return r;
    hipStream_t st = (hipStream_t)stream;
    const int tile = use_mfma ? dm::hard_mfma_block_symbols() : dm::hard_tile_symbols();
    int64_t exact_total = 0;
    for (int s0 = 0; s0 < n_blk; s0 += dm::kMaxSnrPerLaunch) {
        const int nb = std::min(dm::kMaxSnrPerLaunch, n_blk - s0);
        dm::HardArgs a;
        std::memset(&a, 0, sizeof a);
        a.table = c->d_table;
        a.row2label = c->d_row2label;
        a.tx = tx;
        for (int s = 0; s < nb; ++s) {
            a.y[s] = y[s0 + s];
            a.labels_out[s] = labels_out ? labels_out[s0 + s] : nullptr;
        }
        a.N = N;
        a.tiles_per_blk = (N + tile - 1) / tile;
        a.M = c->M;
        a.D = c->D;
        a.n_blk = nb;
        a.counts = counting ? c->d_acc : nullptr;
        a.bad_tx = counting ? c->d_fix_pairs + dm::kMaxSnrPerLaunch : nullptr;
        if (counting) {
            DM_HIP_TRY(hipMemsetAsync(c->d_acc, 0, sizeof(unsigned long long) * 2 * nb, st));
            DM_HIP_TRY(hipMemsetAsync(a.bad_tx, 0, sizeof(uint32_t), st));
        }
        const int64_t work = a.tiles_per_blk * nb;
        if (use_mfma) {
            DM_HIP_TRY(hipMemsetAsync(c->d_queue_count, 0, sizeof(uint32_t), st));
            const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(work, (int64_t)c->cus));
            DM_HIP_TRY(dm::launch_hard_mfma(a, c->d_frag[DM_PREC_FP16X3], std::sqrt(c->max_norm), c->d_queue,
                                            c->d_queue_count, c->queue_cap, grid, st));
            DM_HIP_TRY(dm::launch_hard_fix(a, c->d_queue, c->d_queue_count, c->queue_cap, c->cus * 4, st));
        } else {
            const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(work, (int64_t)c->cus * 2));
            DM_HIP_TRY(dm::launch_hard_demap(a, grid, st));
        }
        if (use_mfma && n_exact) {
            uint32_t q = 0;
            DM_HIP_TRY(hipMemcpyAsync(&q, c->d_queue_count, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
            DM_HIP_TRY(hipStreamSynchronize(st));
            exact_total += q;
        }
        if (counting) {
            auto* h = (unsigned long long*)c->h_stage;
            auto* bad = (uint32_t*)(h + 2 * dm::kMaxSnrPerLaunch);
            DM_HIP_TRY(hipMemcpyAsync(h, c->d_acc, sizeof(unsigned long long) * 2 * nb, hipMemcpyDeviceToHost, st));
            DM_HIP_TRY(hipMemcpyAsync(bad, a.bad_tx, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
            DM_HIP_TRY(hipStreamSynchronize(st));
            if (*bad) return fail(DM_EINVAL, "a transmitted index is >= M");
            for (int s = 0; s < nb; ++s) {
                if (sym_err) sym_err[s0 + s] = (int64_t)h[2 * s];
                if (bit_err) bit_err[s0 + s] = (int64_t)h[2 * s + 1];
            }
        }
    }
    if (n_exact) *n_exact = exact_total;
    return DM_OK;
}

double dm_q_factor_db(double ber) {
    if (!(ber > 0.0) || !(ber < 0.5)) return std::numeric_limits<double>::quiet_NaN();
    // Solve erfc(x) = 2 ber for x > 0 (erfc decreasing): bisection to a bracket, then Newton.
    const double target = 2.0 * ber;
    double lo = 0.0, hi = 1.0;
    while (std::erfc(hi) > target) hi *= 2.0;
    double x = 0.5 * (lo + hi);
    for (int it = 0; it < 200; ++it) {
        const double f = std::erfc(x) - target;
        if (f > 0.0) lo = x;
        else hi = x;
        const double df = -2.0 / std::sqrt(M_PI) * std::exp(-x * x);
        double xn = x - f / df;
        if (!(xn > lo && xn < hi)) xn = 0.5 * (lo + hi);
        if (std::fabs(xn - x) <= 1e-15 * std::max(1.0, x)) {
            x = xn;
            break;
        }
        x = xn;
    }
    return 20.0 * std::log10(std::sqrt(2.0) * x);
}

}  // extern "C"
