// C ABI of the soft-demapping library: validation, constellation upload (label-order
// table), library scratch, kernel launches and the fixed-point GMI / MI finalisation.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/demap.h"
#include "../../include/demap_probe.h"
#include "api_internal.hpp"
#include "device_common.hpp"
#include "kernels.hpp"

using dm::FixEntry;
using dm::LaunchArgs;

namespace dmapi {

thread_local std::string g_err;
thread_local std::vector<int64_t> g_fix_counts;
thread_local bool g_have_fix = false;

// Kernel timing (dm_profile_*): events recorded around each launch on its stream.
struct ProfRec {
    hipEvent_t e0, e1, e2;
};
thread_local bool g_prof_on = false;
thread_local std::vector<ProfRec> g_prof;
thread_local std::vector<hipEvent_t> g_prof_pool;

hipEvent_t prof_event() {
    if (!g_prof_pool.empty()) {
        hipEvent_t e = g_prof_pool.back();
        g_prof_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

void clear_error() { g_err.clear(); }

void forget_fix_counts() {
    g_fix_counts.clear();  // keeps its capacity: no deallocation
    g_have_fix = false;
}

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int hip_fail(hipError_t e, const char* what) {
    return fail(DM_EHIP, "%s failed: %s", what, hipGetErrorString(e));
}


constexpr size_t kStageBytes =
    sizeof(unsigned long long) * dm::kMaxSnrPerLaunch * dm::kAccSlots * 2 + sizeof(uint32_t) * (dm::kMaxSnrPerLaunch + 1);

// Device pointers must be device (or managed) memory of the current device.
int check_device_ptr(const void* p, const char* name, int device) {
    if (!p) return fail(DM_EINVAL, "%s is null", name);
    hipPointerAttribute_t attr;
    hipError_t e = hipPointerGetAttributes(&attr, p);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(DM_EINVAL, "%s is not a device pointer", name);
    }
    if (attr.type != hipMemoryTypeDevice && attr.type != hipMemoryTypeManaged)
        return fail(DM_EINVAL, "%s is not device memory", name);
    if (attr.device != device) return fail(DM_EINVAL, "%s lives on device %d, constellation on %d", name, attr.device, device);
    return DM_OK;
}

int check_current_device(const dm_constellation* c) {
    int dev = -1;
    DM_HIP_TRY(hipGetDevice(&dev));
    if (dev != c->device) return fail(DM_EINVAL, "current device %d differs from the constellation's device %d", dev, c->device);
    return DM_OK;
}

int ensure_scratch(dm_constellation* c, uint64_t want_queue) {
    if (!c->d_acc) {
        DM_HIP_TRY(hipMalloc(&c->d_acc, sizeof(unsigned long long) * dm::kMaxSnrPerLaunch * dm::kAccSlots * 2));
        DM_HIP_TRY(hipMalloc(&c->d_fix_pairs, sizeof(uint32_t) * (dm::kMaxSnrPerLaunch + 1)));
        DM_HIP_TRY(hipMalloc(&c->d_queue_count, sizeof(uint32_t) * dm::kQueueCounterWords));
        DM_HIP_TRY(hipHostMalloc(&c->h_stage, kStageBytes, hipHostMallocDefault));
    }
    const uint64_t cap = std::min<uint64_t>(std::max<uint64_t>(want_queue, 1024), 1u << 22);
    if (cap > c->queue_cap) {
        if (c->d_queue) DM_HIP_TRY(hipFree(c->d_queue));
        c->d_queue = nullptr;
        c->queue_cap = 0;
        if (hipMalloc(&c->d_queue, sizeof(FixEntry) * cap) != hipSuccess) {
            (void)hipGetLastError();
            return fail(DM_ENOMEM, "fix-up queue allocation (%llu entries) failed", (unsigned long long)cap);
        }
        c->queue_cap = (uint32_t)cap;
    }
    return DM_OK;
}

int persistent_grid(const dm_constellation* c, int64_t tiles, int blocks_per_cu) {
    const int64_t g = (int64_t)c->cus * blocks_per_cu;
    return (int)std::max<int64_t>(1, std::min<int64_t>(tiles, g));
}

LaunchArgs base_args(const dm_constellation* c, int64_t N) {
    LaunchArgs a;
    std::memset(&a, 0, sizeof a);
    a.table = c->d_table;
    a.row2label = c->d_row2label;
    a.N = N;
    a.M = c->M;
    a.D = c->D;
    a.m = c->m;
    a.K = (float)(123 - c->m);
    a.flag_thresh = std::ldexp(1.0f, c->m - 102);
    a.near_thresh = std::ldexp(1.0f, c->m - 42);
    return a;
}

uint16_t bf16_bits(float f) {  // round to nearest even
    uint32_t u;
    std::memcpy(&u, &f, 4);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
float bf16_value(uint16_t b) {
    uint32_t u = (uint32_t)b << 16;
    float f;
    std::memcpy(&f, &u, 4);
    return f;
}
uint16_t f16_bits(float f) {
    _Float16 h = (_Float16)f;
    uint16_t b;
    std::memcpy(&b, &h, 2);
    return b;
}
float f16_value(uint16_t b) {
    _Float16 h;
    std::memcpy(&h, &b, 2);
    return (float)h;
}

// Point-side operand table of an MFMA precision in fragment order [tile][mfma][lane][8].
// Row i of a 32-point tile carries label 32t + 16*((i>>2)&1) + 4*(i>>3) + (i&3).
int ensure_frag(dm_constellation* c, int prec, bool pad8) {
    void*& frag_slot = pad8 ? c->d_frag8[prec] : c->d_frag[prec];
    void*& pv_slot = pad8 ? c->d_pv8[prec] : c->d_pv[prec];
    if (frag_slot) return DM_OK;
    const bool bf = (prec == DM_PREC_BF16 || prec == DM_PREC_BF16X3);
    const bool split = (prec == DM_PREC_BF16X3 || prec == DM_PREC_FP16X3);
    const int D = pad8 ? 8 : c->D, M = c->M, Dsrc = c->D;
    const int K = dm::mfma_slots(D, split), S = K / 16;
    auto hi = [&](float v) { return bf ? bf16_bits(v) : f16_bits(v); };
    auto val = [&](uint16_t b) { return bf ? bf16_value(b) : f16_value(b); };
    auto lo = [&](float v) { return hi(v - val(hi(v))); };
    std::vector<uint16_t> pv((size_t)M * K, 0);  // per label, K slots
    for (int l = 0; l < M; ++l) {
        float x[32] = {0.0f};
        for (int d = 0; d < Dsrc; ++d) x[d] = c->h_table[(size_t)l * Dsrc + d];
        double n = 0.0;
        for (int d = 0; d < D; ++d) n += (double)x[d] * (double)x[d];
        const float nn = -(float)n;
        uint16_t* o = &pv[(size_t)l * K];
        if (!split) {
            for (int d = 0; d < D; ++d) o[d] = hi(x[d]);
            o[D] = hi(nn);
            o[D + 1] = hi(1.0f);
        } else {
            for (int d = 0; d < D; ++d) {
                o[d] = hi(x[d]);
                o[D + d] = hi(x[d]);
                o[2 * D + d] = lo(x[d]);
            }
            o[3 * D] = hi(nn);
            o[3 * D + 1] = hi(nn);
            o[3 * D + 2] = lo(nn);
            o[3 * D + 3] = hi(1.0f);
            o[3 * D + 4] = hi(1.0f);
        }
    }
    const int ntiles = M / 32;
    std::vector<uint16_t> fr((size_t)ntiles * S * 64 * 8);
    for (int t = 0; t < ntiles; ++t)
        for (int sidx = 0; sidx < S; ++sidx)
            for (int ln = 0; ln < 64; ++ln) {
                const int i = ln % 32;
                const int label = 32 * t + 16 * ((i >> 2) & 1) + 4 * (i >> 3) + (i & 3);
                const int base = 16 * sidx + 8 * (ln / 32);
                for (int v = 0; v < 8; ++v)
                    fr[(((size_t)t * S + sidx) * 64 + ln) * 8 + v] = pv[(size_t)label * K + base + v];
            }
    void *d = nullptr, *dp = nullptr;
    DM_HIP_TRY(hipMalloc(&d, fr.size() * sizeof(uint16_t)));
    hipError_t e = hipMalloc(&dp, pv.size() * sizeof(uint16_t));
    if (e == hipSuccess) e = hipMemcpy(d, fr.data(), fr.size() * sizeof(uint16_t), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(dp, pv.data(), pv.size() * sizeof(uint16_t), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(d);
        (void)hipFree(dp);
        return hip_fail(e, "fragment table upload");
    }
    frag_slot = d;
    pv_slot = dp;
    return DM_OK;
}

// FP32 label-order table with row stride 8 (batched launches).
int ensure_table8(dm_constellation* c) {
    if (c->d_table8) return DM_OK;
    std::vector<float> t((size_t)c->M * 8, 0.0f);
    for (int l = 0; l < c->M; ++l)
        for (int d = 0; d < c->D; ++d) t[(size_t)l * 8 + d] = c->h_table[(size_t)l * c->D + d];
    DM_HIP_TRY(hipMalloc(&c->d_table8, t.size() * sizeof(float)));
    DM_HIP_TRY(hipMemcpy(c->d_table8, t.data(), t.size() * sizeof(float), hipMemcpyHostToDevice));
    return DM_OK;
}

float exponent_scale(double sigma2) { return (float)(1.4426950408889634 / (2.0 * sigma2)); }

int validate_sigma2(double s2) {
    if (!(s2 > 0.0) || !std::isfinite(s2)) return fail(DM_EINVAL, "sigma2 must be finite and > 0 (got %g)", s2);
    const double c = 1.4426950408889634 / (2.0 * s2);
    if (!(c < 1e30) || !(c > 1e-30)) return fail(DM_EUNSUPPORTED, "sigma2 %g is outside the supported range", s2);
    return DM_OK;
}

// Run the demapper over up to kMaxSnrPerLaunch SNR points of one block, with the accumulators,
// flags and fix-up queue of `scr` (cleared by the caller).  Allocates nothing: an MFMA
// precision needs its operand table already built.
int run_chunk_on(dm_constellation* c, const ChunkScratch& scr, int n_snr, const double* sigma2,
                 const float* const* y, const uint16_t* tx, int64_t N, float* const* llr, bool want_acc, int prec,
                 hipStream_t st, const float* sigma2_sym, bool allow_prof) {
    if (prec != DM_PREC_FP32) {
        if (c->D > 8) return fail(DM_EUNSUPPORTED, "MFMA precisions support D <= 8 (D=%d)", c->D);
        if (c->M < 32) return fail(DM_EUNSUPPORTED, "MFMA precisions need M >= 32 (M=%d)", c->M);
        if (prec == DM_PREC_FP16 || prec == DM_PREC_FP16X3) {
            if (c->max_norm >= 60000.0f) return fail(DM_EUNSUPPORTED, "point norms exceed the FP16 operand range");
            for (int s = 0; s < n_snr; ++s)
                if (exponent_scale(sigma2[s]) >= 30000.0f)
                    return fail(DM_EUNSUPPORTED, "sigma2 %g is too small for FP16 operands", sigma2[s]);
        }
        if (!c->d_frag[prec] || !c->d_pv[prec])
            return fail(DM_EUNSUPPORTED, "the operand table of precision %d is not built for this constellation", prec);
    }
    const int tile = prec == DM_PREC_FP32 ? dm::valu_tile_symbols() : dm::mfma_block_symbols();
    const int64_t tiles_per_snr = (N + tile - 1) / tile;
    LaunchArgs a = base_args(c, N);
    a.tx = tx;
    a.tiles_per_snr = tiles_per_snr;
    a.n_snr = n_snr;
    a.want_llr = llr ? 1 : 0;
    a.sigma2_sym = sigma2_sym;
    a.sinks.acc = want_acc ? scr.acc : nullptr;
    a.sinks.fix_pairs = want_acc ? scr.fix_pairs : nullptr;
    a.sinks.bad_tx = want_acc ? scr.fix_pairs + dm::kMaxSnrPerLaunch : nullptr;
    a.sinks.queue = scr.queue;
    a.sinks.queue_count = scr.queue_count;
    a.sinks.queue_cap = scr.queue_cap;
    for (int s = 0; s < n_snr; ++s) {
        a.snr[s].y = y[s];
        a.snr[s].llr = llr ? llr[s] : nullptr;
        a.snr[s].c = exponent_scale(sigma2[s]);
    }
    const int grid = persistent_grid(c, tiles_per_snr * n_snr, prec == DM_PREC_FP32 ? 2 : 1);
    const int fix_grid = c->cus * dm::fixup_blocks_per_cu(c->M);
    ProfRec pr{nullptr, nullptr, nullptr};
    if (g_prof_on && allow_prof) {
        pr = ProfRec{prof_event(), prof_event(), prof_event()};
        if (pr.e0) DM_HIP_TRY(hipEventRecord(pr.e0, st));
    }
    if (prec == DM_PREC_FP32) DM_HIP_TRY(dm::launch_demap_valu(a, grid, st));
    else DM_HIP_TRY(dm::launch_demap_mfma(a, prec, c->d_frag[prec], c->d_pv[prec], grid, st));
    if (pr.e1) DM_HIP_TRY(hipEventRecord(pr.e1, st));
    DM_HIP_TRY(dm::launch_fixup(a, fix_grid, st));
    if (pr.e2) {
        DM_HIP_TRY(hipEventRecord(pr.e2, st));
        g_prof.push_back(pr);
    }
    return DM_OK;
}

// The same with the constellation's own scratch, grown (and the operand table built) as needed.
int run_chunk(dm_constellation* c, int n_snr, const double* sigma2, const float* const* y, const uint16_t* tx,
              int64_t N, float* const* llr, bool want_acc, int prec, hipStream_t st, const float* sigma2_sym) {
    int r;
    if (prec != DM_PREC_FP32 && c->D <= 8 && c->M >= 32 && (r = ensure_frag(c, prec, false))) return r;
    if ((r = ensure_scratch(c, (uint64_t)N * n_snr))) return r;
    if (want_acc) {
        DM_HIP_TRY(hipMemsetAsync(c->d_acc, 0, sizeof(unsigned long long) * n_snr * dm::kAccSlots * 2, st));
        DM_HIP_TRY(hipMemsetAsync(c->d_fix_pairs, 0, sizeof(uint32_t) * (dm::kMaxSnrPerLaunch + 1), st));
    }
    DM_HIP_TRY(hipMemsetAsync(c->d_queue_count, 0, sizeof(uint32_t) * dm::kQueueCounterWords, st));
    const ChunkScratch scr{c->d_acc, c->d_fix_pairs, c->d_queue_count, c->d_queue, c->queue_cap};
    return run_chunk_on(c, scr, n_snr, sigma2, y, tx, N, llr, want_acc, prec, st, sigma2_sym, true);
}

int llr_var_run(dm_constellation* c, const float* sigma2_sym, const float* y, int64_t N, float* llr, int prec,
                hipStream_t st) {
    std::lock_guard<std::mutex> lock(c->mu);
    const double unit = 1.0;  // replaced per symbol by sigma2_sym
    const float* ys[1] = {y};
    float* ls[1] = {llr};
    return run_chunk(c, 1, &unit, ys, nullptr, N, ls, false, prec, st, sigma2_sym);
}

// Replace the point coordinates of a constellation, given in label order (host, M x D), keeping
// M, D and the labelling; rewrites the device tables in place (same addresses, so plans built
// on c see the new points).  MFMA operand tables are dropped (rebuilt on next use) unless a
// batched copy of them exists, which cannot be rebuilt in place: that case is refused.
int set_label_table(dm_constellation* c, const float* table) {
    std::lock_guard<std::mutex> lock(c->mu);
    for (int p = 0; p < 5; ++p)
        if (c->d_frag8[p]) return fail(DM_EUNSUPPORTED, "constellation has batched MFMA tables; points are fixed");
    float mx = 0.0f;
    for (int l = 0; l < c->M; ++l) {
        double n = 0.0;
        for (int d = 0; d < c->D; ++d) {
            const float v = table[(size_t)l * c->D + d];
            if (!std::isfinite(v) || std::fabs(v) > 1e15f) return fail(DM_EINVAL, "point coordinate is not finite");
            n += (double)v * v;
        }
        mx = std::max(mx, (float)n);
    }
    c->h_table.assign(table, table + (size_t)c->M * c->D);
    c->max_norm = mx;
    c->hash = table_hash(c->M, c->D, c->h_table);
    std::vector<float> padded((size_t)c->M * c->DP, 0.0f);
    for (int l = 0; l < c->M; ++l)
        for (int d = 0; d < c->D; ++d) padded[(size_t)l * c->DP + d] = table[(size_t)l * c->D + d];
    DM_HIP_TRY(hipMemcpy(c->d_table, padded.data(), padded.size() * sizeof(float), hipMemcpyHostToDevice));
    if (c->d_table8) {
        std::vector<float> t8((size_t)c->M * 8, 0.0f);
        for (int l = 0; l < c->M; ++l)
            for (int d = 0; d < c->D; ++d) t8[(size_t)l * 8 + d] = table[(size_t)l * c->D + d];
        DM_HIP_TRY(hipMemcpy(c->d_table8, t8.data(), t8.size() * sizeof(float), hipMemcpyHostToDevice));
    }
    for (int p = 0; p < 5; ++p) {
        if (c->d_frag[p]) (void)hipFree(c->d_frag[p]);
        if (c->d_pv[p]) (void)hipFree(c->d_pv[p]);
        c->d_frag[p] = nullptr;
        c->d_pv[p] = nullptr;
    }
    return DM_OK;
}

// FNV-1a over M, D and the label-order table: identifies the constellation a network was trained on.
uint64_t table_hash(int M, int D, const std::vector<float>& table) {
    uint64_t h = 1469598103934665603ull;
    auto mix = [&](const void* p, size_t n) {
        const unsigned char* b = (const unsigned char*)p;
        for (size_t i = 0; i < n; ++i) {
            h ^= b[i];
            h *= 1099511628211ull;
        }
    };
    mix(&M, sizeof M);
    mix(&D, sizeof D);
    mix(table.data(), table.size() * sizeof(float));
    return h;
}

}  // namespace dmapi

using namespace dmapi;

extern "C" {

const char* dm_last_error(void) { return g_err.c_str(); }

const char* dm_version(void) { return "demap-mi355x 0.1 (gfx950)"; }

int dm_constellation_create(const float* points, const uint16_t* labels, int32_t M, int32_t D,
                            dm_constellation** out) {
    g_err.clear();
    if (!points || !labels || !out) return fail(DM_EINVAL, "null argument");
    *out = nullptr;
    if (M < 2 || (M & (M - 1))) return fail(DM_EINVAL, "M=%d is not a power of two >= 2", M);
    int m = 0;
    while ((1 << m) < M) ++m;
    if (m > 16) return fail(DM_EUNSUPPORTED, "m=%d > 16", m);
    if (D < 1) return fail(DM_EINVAL, "D=%d < 1", D);
    if (D > 32) return fail(DM_EUNSUPPORTED, "D=%d > 32", D);
    std::vector<int> row_of(M, -1);
    for (int j = 0; j < M; ++j) {
        if (labels[j] >= (uint32_t)M || row_of[labels[j]] >= 0)
            return fail(DM_EINVAL, "labels are not a bijection onto [0, M) (row %d)", j);
        row_of[labels[j]] = j;
    }
    for (size_t i = 0; i < (size_t)M * D; ++i)
        if (!std::isfinite(points[i]) || std::fabs(points[i]) > 1e15f)
            return fail(DM_EINVAL, "point coordinate %zu is not finite or exceeds 1e15", i);

    auto* c = new (std::nothrow) dm_constellation();
    if (!c) return fail(DM_ENOMEM, "host allocation failed");
    c->M = M;
    c->D = D;
    c->m = m;
    c->DP = dm::padded_dim(D);
    hipError_t e = hipGetDevice(&c->device);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&c->cus, hipDeviceAttributeMultiprocessorCount, c->device);
    if (e != hipSuccess) {
        delete c;
        return hip_fail(e, "device query");
    }
    c->h_table.assign((size_t)M * D, 0.0f);
    for (int j = 0; j < M; ++j) {
        double n = 0.0;
        for (int d = 0; d < D; ++d) n += (double)points[(size_t)j * D + d] * points[(size_t)j * D + d];
        c->max_norm = std::max(c->max_norm, (float)n);
    }
    std::vector<float> padded((size_t)M * c->DP, 0.0f);
    std::vector<uint16_t> r2l(labels, labels + M);
    for (int l = 0; l < M; ++l)
        for (int d = 0; d < D; ++d) {
            c->h_table[(size_t)l * D + d] = points[(size_t)row_of[l] * D + d];
            padded[(size_t)l * c->DP + d] = points[(size_t)row_of[l] * D + d];
        }
    c->hash = table_hash(M, D, c->h_table);
    if ((e = hipMalloc(&c->d_table, padded.size() * sizeof(float))) != hipSuccess ||
        (e = hipMalloc(&c->d_row2label, M * sizeof(uint16_t))) != hipSuccess ||
        (e = hipMemcpy(c->d_table, padded.data(), padded.size() * sizeof(float), hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(c->d_row2label, r2l.data(), M * sizeof(uint16_t), hipMemcpyHostToDevice)) != hipSuccess) {
        dm_constellation_destroy(c);
        return hip_fail(e, "constellation upload");
    }
    // MFMA operand tables of every precision are built here, once, so that later calls (the
    // allocation-free GMI entry point among them) find them ready.
    if (M >= 32 && D <= 8)
        for (int prec = DM_PREC_BF16; prec <= DM_PREC_FP16X3; ++prec) {
            const int r = ensure_frag(c, prec, false);
            if (r) {
                dm_constellation_destroy(c);
                return r;
            }
        }
    *out = c;
    return DM_OK;
}

void dm_constellation_destroy(dm_constellation* c) {
    if (!c) return;
    (void)hipFree(c->d_table);
    (void)hipFree(c->d_row2label);
    (void)hipFree(c->d_acc);
    (void)hipFree(c->d_fix_pairs);
    (void)hipFree(c->d_queue_count);
    (void)hipFree(c->d_queue);
    if (c->h_stage) (void)hipHostFree(c->h_stage);
    for (void* f : c->d_frag) (void)hipFree(f);
    for (void* f : c->d_pv) (void)hipFree(f);
    for (void* f : c->d_frag8) (void)hipFree(f);
    for (void* f : c->d_pv8) (void)hipFree(f);
    (void)hipFree(c->d_table8);
    delete c;
}

int dm_demap_llr(const dm_constellation* cc, double sigma2, const float* y, int64_t N, float* llr, int prec,
                 void* stream) {
    g_err.clear();
    auto* c = const_cast<dm_constellation*>(cc);
    if (!c) return fail(DM_EINVAL, "constellation is null");
    if (N < 0 || N >= (int64_t(1) << 31)) return fail(DM_EINVAL, "N=%lld out of range", (long long)N);
    if (prec < DM_PREC_FP32 || prec > DM_PREC_FP16X3) return fail(DM_EINVAL, "unknown precision %d", prec);
    int r = validate_sigma2(sigma2);
    if (r) return r;
    if (N == 0) return DM_OK;
    if ((r = check_current_device(c))) return r;
    if ((r = check_device_ptr(y, "y", c->device))) return r;
    if ((r = check_device_ptr(llr, "llr", c->device))) return r;
    std::lock_guard<std::mutex> lock(c->mu);
    const float* ys[1] = {y};
    float* ls[1] = {llr};
    return run_chunk(c, 1, &sigma2, ys, nullptr, N, ls, false, prec, (hipStream_t)stream, nullptr);
}

int dm_gmi_estimate(const dm_constellation* cc, int n_snr, const double* sigma2, const float* const* y,
                    const uint16_t* tx, int64_t N, float* const* llr, double* gmi, double* mi, int prec,
                    void* stream) {
    g_err.clear();
    auto* c = const_cast<dm_constellation*>(cc);
    if (!c || !sigma2 || !y || !gmi) return fail(DM_EINVAL, "null argument");
    if (n_snr < 1) return fail(DM_EINVAL, "n_snr=%d < 1", n_snr);
    if (N < 0 || N >= (int64_t(1) << 31)) return fail(DM_EINVAL, "N=%lld out of range", (long long)N);
    if (prec < DM_PREC_FP32 || prec > DM_PREC_FP16X3) return fail(DM_EINVAL, "unknown precision %d", prec);
    int r;
    for (int s = 0; s < n_snr; ++s)
        if ((r = validate_sigma2(sigma2[s]))) return r;
    g_fix_counts.assign(n_snr, 0);
    g_have_fix = true;
    if (N == 0) {
        for (int s = 0; s < n_snr; ++s) {
            gmi[s] = NAN;
            if (mi) mi[s] = NAN;
        }
        return DM_OK;
    }
    if ((r = check_current_device(c))) return r;
    if ((r = check_device_ptr(tx, "tx", c->device))) return r;
    for (int s = 0; s < n_snr; ++s) {
        if ((r = check_device_ptr(y[s], "y[s]", c->device))) return r;
        if (llr && (r = check_device_ptr(llr[s], "llr[s]", c->device))) return r;
    }
    return gmi_run(c, n_snr, sigma2, y, tx, N, llr, gmi, mi, prec, (hipStream_t)stream);
}

}  // extern "C"

namespace dmapi {

int gmi_run(dm_constellation* c, int n_snr, const double* sigma2, const float* const* y, const uint16_t* tx,
            int64_t N, float* const* llr, double* gmi, double* mi, int prec, hipStream_t st) {
    int r;
    std::lock_guard<std::mutex> lock(c->mu);
    for (int s0 = 0; s0 < n_snr; s0 += dm::kMaxSnrPerLaunch) {
        const int ns = std::min(dm::kMaxSnrPerLaunch, n_snr - s0);
        r = run_chunk(c, ns, sigma2 + s0, y + s0, tx, N, llr ? llr + s0 : nullptr, true, prec, st, nullptr);
        if (r) return r;
        auto* acc = (unsigned long long*)c->h_stage;
        auto* fix = (uint32_t*)(acc + (size_t)dm::kMaxSnrPerLaunch * dm::kAccSlots * 2);
        DM_HIP_TRY(hipMemcpyAsync(acc, c->d_acc, sizeof(unsigned long long) * ns * dm::kAccSlots * 2, hipMemcpyDeviceToHost, st));
        DM_HIP_TRY(hipMemcpyAsync(fix, c->d_fix_pairs, sizeof(uint32_t) * (dm::kMaxSnrPerLaunch + 1), hipMemcpyDeviceToHost, st));
        DM_HIP_TRY(hipStreamSynchronize(st));
        if (fix[dm::kMaxSnrPerLaunch]) return fail(DM_EINVAL, "a transmitted index is >= M");
        for (int s = 0; s < ns; ++s) {
            long long gs = 0, ms = 0;  // two's-complement sums of the fixed-point slots
            for (int k = 0; k < dm::kAccSlots; ++k) {
                gs += (long long)acc[((size_t)s * dm::kAccSlots + k) * 2 + 0];
                ms += (long long)acc[((size_t)s * dm::kAccSlots + k) * 2 + 1];
            }
            gmi[s0 + s] = (double)gs / dm::kFixScale / (double)N;
            if (mi) mi[s0 + s] = (double)ms / dm::kFixScale / (double)N;
            if ((size_t)(s0 + s) < g_fix_counts.size()) g_fix_counts[s0 + s] = fix[s];
        }
    }
    return DM_OK;
}

}  // namespace dmapi

extern "C" {

int dm_demap_llr_var(const dm_constellation* cc, const float* sigma2, const float* y, int64_t N, float* llr,
                     int prec, void* stream) {
    g_err.clear();
    auto* c = const_cast<dm_constellation*>(cc);
    if (!c) return fail(DM_EINVAL, "constellation is null");
    if (N < 0 || N >= (int64_t(1) << 31)) return fail(DM_EINVAL, "N=%lld out of range", (long long)N);
    if (prec != DM_PREC_FP32 && prec != DM_PREC_BF16 && prec != DM_PREC_BF16X3)
        return fail(DM_EUNSUPPORTED, "per-symbol noise variances need an FP32-range precision (FP32, BF16, BF16X3)");
    if (N == 0) return DM_OK;
    int r;
    if ((r = check_current_device(c))) return r;
    if ((r = check_device_ptr(sigma2, "sigma2", c->device))) return r;
    if ((r = check_device_ptr(y, "y", c->device))) return r;
    if ((r = check_device_ptr(llr, "llr", c->device))) return r;
    return llr_var_run(c, sigma2, y, N, llr, prec, (hipStream_t)stream);
}

int dm_profile_enable(int on) {
    g_prof_on = on != 0;
    if (g_prof_on) {
        for (auto& r : g_prof) {
            (void)hipEventSynchronize(r.e2);
            g_prof_pool.push_back(r.e0);
            g_prof_pool.push_back(r.e1);
            g_prof_pool.push_back(r.e2);
        }
        g_prof.clear();
    }
    return DM_OK;
}

int dm_profile_read(double* main_ms, double* fixup_ms, int64_t* launches, int reset) {
    double a = 0.0, b = 0.0;
    for (auto& r : g_prof) {
        DM_HIP_TRY(hipEventSynchronize(r.e2));
        float t1 = 0.0f, t2 = 0.0f;
        DM_HIP_TRY(hipEventElapsedTime(&t1, r.e0, r.e1));
        DM_HIP_TRY(hipEventElapsedTime(&t2, r.e1, r.e2));
        a += t1;
        b += t2;
    }
    if (main_ms) *main_ms = a;
    if (fixup_ms) *fixup_ms = b;
    if (launches) *launches = (int64_t)g_prof.size();
    if (reset) {
        for (auto& r : g_prof) {
            g_prof_pool.push_back(r.e0);
            g_prof_pool.push_back(r.e1);
            g_prof_pool.push_back(r.e2);
        }
        g_prof.clear();
    }
    return DM_OK;
}

int64_t dm_last_fixup_count(int64_t* per_snr, int n_snr) {
    if (!g_have_fix) return DM_EINVAL;
    int64_t total = 0;
    for (size_t s = 0; s < g_fix_counts.size(); ++s) {
        total += g_fix_counts[s];
        if (per_snr && (int)s < n_snr) per_snr[s] = g_fix_counts[s];
    }
    return total;
}

}  // extern "C"
