// Streamed demapping of host-resident blocks (the paper's receiver processes fixed-size sample
// buffers as they arrive, Sec. 2): the host block is cut into buffers of B symbols that cycle
// through a ring of n slots, each slot holding pinned host staging (y in, LLRs out) and device
// buffers.  Per buffer: the host copies y into the slot's pinned staging, a copy stream moves it
// to the device, the compute stream demaps it once the copy's event has fired, and a third
// stream moves the LLRs back after the demapping's event; the host collects a slot's LLRs when
// the slot comes round again.  Copies of one buffer thus overlap the demapping of another.
// Page-locked caller arrays are transferred directly, without the staging copies.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <mutex>
#include <vector>

#include "api_internal.hpp"

namespace {

using dmapi::fail;
using dmapi::hip_fail;

struct Slot {
    float* h_y = nullptr;
    float* h_llr = nullptr;
    float* d_y = nullptr;
    float* d_llr = nullptr;
    hipEvent_t in = nullptr, done = nullptr, out = nullptr;
    int64_t first = -1, count = 0;  // symbols of the buffer in flight in this slot (-1: none)
};

}  // namespace

struct dm_streamer {
    dm_constellation* c = nullptr;
    int64_t B = 0;
    int prec = 0;
    std::vector<Slot> slots;
    hipStream_t s_in = nullptr, s_compute = nullptr, s_out = nullptr;
    std::mutex mu;
};

namespace {

void release(dm_streamer* s) {
    for (Slot& q : s->slots) {
        if (q.h_y) (void)hipHostFree(q.h_y);
        if (q.h_llr) (void)hipHostFree(q.h_llr);
        if (q.d_y) (void)hipFree(q.d_y);
        if (q.d_llr) (void)hipFree(q.d_llr);
        for (hipEvent_t e : {q.in, q.done, q.out})
            if (e) (void)hipEventDestroy(e);
    }
    for (hipStream_t st : {s->s_in, s->s_compute, s->s_out})
        if (st) (void)hipStreamDestroy(st);
}

// Copy the finished LLRs of slot q to the caller's array (waits for its D2H copy); with a
// pinned caller array the D2H copy already landed there.
int collect(dm_streamer* s, Slot& q, float* llr, bool direct) {
    if (q.first < 0) return DM_OK;
    DM_HIP_TRY(hipEventSynchronize(q.out));
    if (!direct) std::memcpy(llr + (size_t)q.first * s->c->m, q.h_llr, sizeof(float) * (size_t)q.count * s->c->m);
    q.first = -1;
    return DM_OK;
}

// True when p is page-locked host memory (hipHostMalloc / pinned tensors): DMA can use it as is.
bool pinned(const void* p) {
    hipPointerAttribute_t a;
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return a.type == hipMemoryTypeHost;
}

}  // namespace

extern "C" {

int dm_streamer_create(const dm_constellation* cc, int64_t buffer_symbols, int32_t n_buffers, int32_t prec,
                       dm_streamer** out) {
    dmapi::clear_error();
    auto* c = const_cast<dm_constellation*>(cc);
    if (!c || !out) return fail(DM_EINVAL, "null argument");
    *out = nullptr;
    if (buffer_symbols < 1 || buffer_symbols > (int64_t(1) << 26))
        return fail(DM_EINVAL, "buffer_symbols=%lld outside [1, 2^26]", (long long)buffer_symbols);
    if (n_buffers < 2 || n_buffers > 16) return fail(DM_EINVAL, "n_buffers=%d outside [2, 16]", n_buffers);
    if (prec < DM_PREC_FP32 || prec > DM_PREC_FP16X3) return fail(DM_EINVAL, "unknown precision %d", prec);
    int r = dmapi::check_current_device(c);
    if (r) return r;
    auto* s = new (std::nothrow) dm_streamer();
    if (!s) return fail(DM_ENOMEM, "host allocation failed");
    s->c = c;
    s->B = buffer_symbols;
    s->prec = prec;
    s->slots.resize(n_buffers);
    const size_t ybytes = sizeof(float) * (size_t)buffer_symbols * c->D;
    const size_t lbytes = sizeof(float) * (size_t)buffer_symbols * c->m;
    hipError_t e = hipSuccess;
    for (hipStream_t* st : {&s->s_in, &s->s_compute, &s->s_out})
        if (e == hipSuccess) e = hipStreamCreateWithFlags(st, hipStreamNonBlocking);
    for (Slot& q : s->slots) {
        if (e == hipSuccess) e = hipHostMalloc((void**)&q.h_y, ybytes, hipHostMallocDefault);
        if (e == hipSuccess) e = hipHostMalloc((void**)&q.h_llr, lbytes, hipHostMallocDefault);
        if (e == hipSuccess) e = hipMalloc((void**)&q.d_y, ybytes);
        if (e == hipSuccess) e = hipMalloc((void**)&q.d_llr, lbytes);
        for (hipEvent_t* ev : {&q.in, &q.done, &q.out})
            if (e == hipSuccess) e = hipEventCreateWithFlags(ev, hipEventDisableTiming);
    }
    if (e != hipSuccess) {
        release(s);
        delete s;
        return hip_fail(e, "streamer allocation");
    }
    *out = s;
    return DM_OK;
}

void dm_streamer_destroy(dm_streamer* s) {
    if (!s) return;
    (void)hipDeviceSynchronize();
    release(s);
    delete s;
}

int dm_streamer_run(dm_streamer* s, double sigma2, const float* y, int64_t N, float* llr, double* seconds) {
    dmapi::clear_error();
    if (!s || (N > 0 && (!y || !llr))) return fail(DM_EINVAL, "null argument");
    if (N < 0) return fail(DM_EINVAL, "N < 0");
    int r = dmapi::validate_sigma2(sigma2);
    if (r) return r;
    std::lock_guard<std::mutex> lock(s->mu);
    const auto t0 = std::chrono::steady_clock::now();
    const int D = s->c->D, m = s->c->m;
    const int n = (int)s->slots.size();
    const bool direct_in = N > 0 && pinned(y), direct_out = N > 0 && pinned(llr);
    int64_t k = 0;
    for (int64_t first = 0; first < N; first += s->B, ++k) {
        Slot& q = s->slots[k % n];
        if ((r = collect(s, q, llr, direct_out))) return r;  // the slot's previous buffer is back
        const int64_t cnt = std::min<int64_t>(s->B, N - first);
        const float* src = y + (size_t)first * D;
        if (!direct_in) {
            std::memcpy(q.h_y, src, sizeof(float) * (size_t)cnt * D);
            src = q.h_y;
        }
        DM_HIP_TRY(hipMemcpyAsync(q.d_y, src, sizeof(float) * (size_t)cnt * D, hipMemcpyHostToDevice, s->s_in));
        DM_HIP_TRY(hipEventRecord(q.in, s->s_in));
        DM_HIP_TRY(hipStreamWaitEvent(s->s_compute, q.in, 0));
        if ((r = dm_demap_llr(s->c, sigma2, q.d_y, cnt, q.d_llr, s->prec, s->s_compute))) return r;
        DM_HIP_TRY(hipEventRecord(q.done, s->s_compute));
        DM_HIP_TRY(hipStreamWaitEvent(s->s_out, q.done, 0));
        float* dst = direct_out ? llr + (size_t)first * m : q.h_llr;
        DM_HIP_TRY(hipMemcpyAsync(dst, q.d_llr, sizeof(float) * (size_t)cnt * m, hipMemcpyDeviceToHost, s->s_out));
        DM_HIP_TRY(hipEventRecord(q.out, s->s_out));
        q.first = first;
        q.count = cnt;
    }
    for (Slot& q : s->slots)
        if ((r = collect(s, q, llr, direct_out))) return r;
    if (seconds) *seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return DM_OK;
}

}  // extern "C"
