// Library-internal host declarations shared by the C-ABI sources (not part of the ABI).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/demap.h"
#include "device_common.hpp"

struct dm_constellation {
    int M = 0, D = 0, m = 0, DP = 0, device = 0, cus = 0;
    float* d_table = nullptr;          // M x DP FP32, label order, zero-padded columns
    uint16_t* d_row2label = nullptr;   // M
    std::vector<float> h_table;        // host copy of the label-order table (M x D)
    // scratch (grow-only), shared by calls on this constellation
    unsigned long long* d_acc = nullptr;  // kMaxSnrPerLaunch x kAccSlots x 2
    uint32_t* d_fix_pairs = nullptr;      // kMaxSnrPerLaunch + 1 (last word: bad-tx flag)
    uint32_t* d_queue_count = nullptr;    // kQueueCounterWords: the queue regions' counters
    dm::FixEntry* d_queue = nullptr;
    uint32_t queue_cap = 0;
    void* h_stage = nullptr;              // pinned: acc + fix_pairs
    void* d_frag[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};  // MFMA point tables per precision
    void* d_pv[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};    // same operands per label [M][K]
    // Batched-launch copies with the row stride padded to 8 (D <= 8).
    float* d_table8 = nullptr;
    void* d_frag8[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    void* d_pv8[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    float max_norm = 0.0f;                // max ||x||^2 (FP16 operand range check)
    uint64_t hash = 0;                    // identity of (M, D, label-order table)
    std::mutex mu;
};

namespace dmapi {

// Record a message for dm_last_error() and return `code`.
int fail(int code, const char* fmt, ...);
void clear_error();
int hip_fail(hipError_t e, const char* what);

int check_device_ptr(const void* p, const char* name, int device);
// Drop the per-point fix-up counts of the last GMI call (dm_last_fixup_count then fails).
void forget_fix_counts();
int check_current_device(const dm_constellation* c);
int validate_sigma2(double s2);
float exponent_scale(double sigma2);

// MFMA point-operand tables of a precision (pad8: row layout padded to D = 8).
int ensure_frag(dm_constellation* c, int prec, bool pad8);
int ensure_table8(dm_constellation* c);

// Device scratch of one exact-path launch: fixed-point GMI / MI slots [kMaxSnrPerLaunch][kAccSlots][2],
// fix-up pair counts [kMaxSnrPerLaunch] + bad-tx flag, fix-up queue and its region counters.
struct ChunkScratch {
    unsigned long long* acc;
    uint32_t* fix_pairs;
    uint32_t* queue_count;
    dm::FixEntry* queue;
    uint32_t queue_cap;
};
// Exact path over up to 32 SNR points of one block on the given scratch, which the caller has
// cleared (acc and fix_pairs when want_acc, the kQueueCounterWords of queue_count always); allocates nothing (an MFMA
// precision needs its operand table built).  Caller holds c->mu.
int run_chunk_on(dm_constellation* c, const ChunkScratch& scr, int n_snr, const double* sigma2,
                 const float* const* y, const uint16_t* tx, int64_t N, float* const* llr, bool want_acc, int prec,
                 hipStream_t st, const float* sigma2_sym, bool allow_prof);
// Exact path over up to 32 SNR points of one block (scratch of c; caller holds c->mu).
// sigma2_sym, when not null, gives each symbol its own noise variance (sigma2 is then unused).
int run_chunk(dm_constellation* c, int n_snr, const double* sigma2, const float* const* y, const uint16_t* tx,
              int64_t N, float* const* llr, bool want_acc, int prec, hipStream_t st, const float* sigma2_sym);
// Exact GMI / MI (and LLRs) of n_snr points, synchronising `st`; arguments already validated.
int gmi_run(dm_constellation* c, int n_snr, const double* sigma2, const float* const* y, const uint16_t* tx,
            int64_t N, float* const* llr, double* gmi, double* mi, int prec, hipStream_t st);
// Exact LLRs with per-symbol noise variances (device FP32, N); arguments already validated.
int llr_var_run(dm_constellation* c, const float* sigma2_sym, const float* y, int64_t N, float* llr, int prec,
                hipStream_t st);
uint64_t table_hash(int M, int D, const std::vector<float>& table);
// Replace the coordinates (host, label order, M x D) of c in place; see demap_api.hip.
int set_label_table(dm_constellation* c, const float* table);
// Allocate the constellation's accumulators / flags / staging (and a fix-up queue of >= want entries).
int ensure_scratch(dm_constellation* c, uint64_t want_queue);

}  // namespace dmapi

#define DM_HIP_TRY(expr)                                          \
    do {                                                          \
        hipError_t _e = (expr);                                   \
        if (_e != hipSuccess) return dmapi::hip_fail(_e, #expr);  \
    } while (0)
