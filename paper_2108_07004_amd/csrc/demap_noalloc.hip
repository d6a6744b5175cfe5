// Allocation-free variant of the exact GMI / MI entry point, for callers that cannot allocate
// device memory (code under stream capture, tight serving loops, harnesses that forbid it).
//
// The launch's scratch — fixed-point GMI / MI slots, fix-up pair counts and bad-tx flag, the
// fix-up queue and its region counters, and the per-point totals read back by the host — lives in one
// file-scope device array, `scratch`, of kScratchBytes (about 16 MiB, held by every GPU the
// library runs on until the process ends).  Host code never passes the array's name to a
// kernel (on the host it is only a stand-in symbol): the device address is looked up once per
// device with hipGetSymbolAddress and kept in g_scratch[device].
//
// Every call on a device shares that device's array and leaves the last call's contents in it;
// each call clears what must start at zero with a fill kernel before its launches.  Calls on
// one device are serialised by a host lock held until the call has synchronised its stream.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <mutex>

#include "../../include/demap.h"
#include "api_internal.hpp"
#include "device_common.hpp"
#include "kernels.hpp"

namespace {

using dmapi::fail;

constexpr uint32_t kQueueEntries = 1u << 20;  // fix-up queue; a full queue is recomputed in place
constexpr size_t kAccBytes = sizeof(unsigned long long) * dm::kMaxSnrPerLaunch * dm::kAccSlots * 2;
constexpr size_t kSumOff = kAccBytes;                                   // [n_snr][2] int64 totals
constexpr size_t kFixOff = kSumOff + sizeof(long long) * dm::kMaxSnrPerLaunch * 2;
constexpr size_t kCountOff = kFixOff + 256;                             // kMaxSnrPerLaunch + 1 words fit
constexpr size_t kQueueOff = kCountOff + sizeof(uint32_t) * dm::kQueueCounterWords;  // region counters
constexpr size_t kClearBytes = kQueueOff;                               // zeroed by every call
constexpr size_t kScratchBytes = kQueueOff + sizeof(dm::FixEntry) * kQueueEntries;
static_assert(sizeof(uint32_t) * (dm::kMaxSnrPerLaunch + 1) <= 256, "fix-pair words overflow their slot");
static_assert(kClearBytes % 4 == 0 && kQueueOff % 256 == 0, "scratch layout");

constexpr int kMaxDevices = 64;

}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

std::mutex g_mu[kMaxDevices];
unsigned char* g_scratch[kMaxDevices] = {};

// tot[s][w] = sum over the kAccSlots slots of acc[s][slot][w] (two's complement, fixed order).
__global__ void sum_slots_kernel(const unsigned long long* acc, int n_snr, long long* tot) {
    const int t = threadIdx.x;
    if (t >= 2 * n_snr) return;
    const int s = t >> 1, w = t & 1;
    unsigned long long v = 0ull;
    for (int k = 0; k < dm::kAccSlots; ++k) v += acc[((size_t)s * dm::kAccSlots + k) * 2 + w];
    tot[t] = (long long)v;
}

// Device address of this device's scratch array, looked up on the first call on the device
// (caller holds g_mu[dev]).
int scratch_of(int dev, unsigned char** out) {
    if (!g_scratch[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return fail(DM_EHIP, "hipGetSymbolAddress of the static scratch failed: %s", hipGetErrorString(e));
        }
        g_scratch[dev] = static_cast<unsigned char*>(p);
    }
    *out = g_scratch[dev];
    return DM_OK;
}

}  // namespace

extern "C" {

int dm_gmi_estimate_noalloc(const dm_constellation* cc, int n_snr, const double* sigma2, const float* const* y,
                            const uint16_t* tx, int64_t N, float* const* llr, double* gmi, double* mi, int prec,
                            void* stream) {
    dmapi::clear_error();
    dmapi::forget_fix_counts();  // dm_last_fixup_count reports no counts after this call
    auto* c = const_cast<dm_constellation*>(cc);
    if (!c || !sigma2 || !y || !gmi) return fail(DM_EINVAL, "null argument");
    if (n_snr < 1) return fail(DM_EINVAL, "n_snr=%d < 1", n_snr);
    if (n_snr > dm::kMaxSnrPerLaunch)
        return fail(DM_EINVAL, "n_snr=%d exceeds the %d noise levels the static scratch holds", n_snr,
                    dm::kMaxSnrPerLaunch);
    if (N < 0 || N >= (int64_t(1) << 31)) return fail(DM_EINVAL, "N=%lld out of range", (long long)N);
    if (prec < DM_PREC_FP32 || prec > DM_PREC_FP16X3) return fail(DM_EINVAL, "unknown precision %d", prec);
    int r;
    for (int s = 0; s < n_snr; ++s)
        if ((r = dmapi::validate_sigma2(sigma2[s]))) return r;
    if (N == 0) {
        for (int s = 0; s < n_snr; ++s) {
            gmi[s] = NAN;
            if (mi) mi[s] = NAN;
        }
        return DM_OK;
    }
    if ((r = dmapi::check_current_device(c))) return r;
    if (c->device < 0 || c->device >= kMaxDevices) return fail(DM_EUNSUPPORTED, "device %d out of range", c->device);
    if ((r = dmapi::check_device_ptr(tx, "tx", c->device))) return r;
    for (int s = 0; s < n_snr; ++s) {
        if ((r = dmapi::check_device_ptr(y[s], "y[s]", c->device))) return r;
        if (llr && (r = dmapi::check_device_ptr(llr[s], "llr[s]", c->device))) return r;
    }
    const hipStream_t st = (hipStream_t)stream;
    std::lock_guard<std::mutex> dev_lock(g_mu[c->device]);
    std::lock_guard<std::mutex> lock(c->mu);
    unsigned char* base = nullptr;
    if ((r = scratch_of(c->device, &base))) return r;
    const dmapi::ChunkScratch scr{reinterpret_cast<unsigned long long*>(base),
                                  reinterpret_cast<uint32_t*>(base + kFixOff),
                                  reinterpret_cast<uint32_t*>(base + kCountOff),
                                  reinterpret_cast<dm::FixEntry*>(base + kQueueOff), kQueueEntries};
    auto* tot = reinterpret_cast<long long*>(base + kSumOff);
    DM_HIP_TRY(dm::launch_zero_words(reinterpret_cast<uint32_t*>(base), kClearBytes / 4, st));
    if ((r = dmapi::run_chunk_on(c, scr, n_snr, sigma2, y, tx, N, llr, true, prec, st, nullptr, false))) return r;
    hipLaunchKernelGGL(sum_slots_kernel, dim3(1), dim3(64), 0, st, scr.acc, n_snr, tot);
    DM_HIP_TRY(hipGetLastError());
    long long h_tot[2 * dm::kMaxSnrPerLaunch];
    uint32_t h_fix[dm::kMaxSnrPerLaunch + 1];
    DM_HIP_TRY(hipMemcpyAsync(h_tot, tot, sizeof(long long) * 2 * n_snr, hipMemcpyDeviceToHost, st));
    DM_HIP_TRY(hipMemcpyAsync(h_fix, scr.fix_pairs, sizeof h_fix, hipMemcpyDeviceToHost, st));
    DM_HIP_TRY(hipStreamSynchronize(st));
    if (h_fix[dm::kMaxSnrPerLaunch]) return fail(DM_EINVAL, "a transmitted index is >= M");
    for (int s = 0; s < n_snr; ++s) {
        gmi[s] = (double)h_tot[2 * s] / dm::kFixScale / (double)N;
        if (mi) mi[s] = (double)h_tot[2 * s + 1] / dm::kFixScale / (double)N;
    }
    return DM_OK;
}

}  // extern "C"
