// Batched demapping plans: one persistent launch over many instances of uneven M, D and N,
// an autotuner that picks the launch shape by timing, a work list that workgroups claim chunk
// by chunk from a device counter at run time, and a hipGraph that replays zero-fill + batched
// kernel + fix-up with one launch.
//
// Shape of a plan: per (M, D, precision) class the kernel body (FP32 direct differences or MFMA
// cross terms) and the work-item size (1, 2 or 4 of the body's symbol tiles: larger items pay
// the per-item descriptor reads and wave reductions less often, smaller ones balance the tail
// better); per plan the claim size (1, 2, 4 or 8 work items per counter increment).  The
// autotuner times every body x item size of a class on a replicated probe block large enough
// to fill the GPU (cached per GPU arch), then the whole plan at each claim size.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/demap.h"
#include "api_internal.hpp"
#include "device_common.hpp"
#include "kernels.hpp"

using namespace dmapi;

namespace {

constexpr int kGrabDefault = 4;       // work items per claim without autotuning
constexpr int kSubs[] = {1, 2, 4};    // item sizes (symbol tiles per work item) tried per class
constexpr int kGrabs[] = {1, 2, 4, 8};  // claim sizes tried per plan
constexpr int kProbeItemsPerCu = 4;   // probe block: this many work items per CU
constexpr int kProbeCopies = 64;      // at most this many copies of the probe instance

struct TuneKey {
    int M, D, prec, kind, sub;
    bool operator<(const TuneKey& o) const {
        return std::tie(M, D, prec, kind, sub) < std::tie(o.M, o.D, o.prec, o.kind, o.sub);
    }
};

std::mutex g_tune_mu;
std::map<TuneKey, double> g_tune;  // ns per (symbol, point) pair
bool g_tune_loaded = false;

std::string tune_cache_path() {
    const char* p = std::getenv("DM_AUTOTUNE_CACHE");
    return p ? std::string(p) : std::string();
}

std::string arch_name() {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
    std::string a = prop.gcnArchName;
    const size_t colon = a.find(':');
    return colon == std::string::npos ? a : a.substr(0, colon);
}

// Cache file: one line per entry, "shape2 arch M D prec kind sub ns_per_pair" (lines of any
// other format are ignored).
void load_tune_cache() {
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const std::string path = tune_cache_path();
    if (path.empty()) return;
    std::ifstream f(path);
    const std::string arch = arch_name();
    std::string line;
    while (std::getline(f, line)) {
        std::istringstream in(line);
        std::string tag, a;
        TuneKey k;
        double v;
        if (in >> tag >> a >> k.M >> k.D >> k.prec >> k.kind >> k.sub >> v && tag == "shape2" && a == arch && v > 0.0)
            g_tune[k] = v;
    }
}

void save_tune_cache() {
    const std::string path = tune_cache_path();
    if (path.empty()) return;
    std::ofstream f(path, std::ios::trunc);
    const std::string arch = arch_name();
    for (const auto& kv : g_tune)
        f << "shape2 " << arch << ' ' << kv.first.M << ' ' << kv.first.D << ' ' << kv.first.prec << ' '
          << kv.first.kind << ' ' << kv.first.sub << ' ' << kv.second << '\n';
}

bool mfma_possible(const dm_constellation* c, int prec) {
    if (prec == DM_PREC_FP32 || c->M < 32 || c->D > 8) return false;
    const bool split = (prec == DM_PREC_BF16X3 || prec == DM_PREC_FP16X3);
    const int S = dm::mfma_slots(8, split) / 16;
    return (size_t)(c->M / 32) * S * 1024 <= (size_t)dm::kBatchedLdsBytes;
}

}  // namespace

struct dm_plan {
    int n_inst = 0, prec = 0, grid = 0, fix_grid = 0, device = 0, grab = 0;
    std::vector<dm_instance> inst;
    std::vector<int> kind;
    std::vector<int> sub;  // symbol tiles per work item
    std::vector<double> ns_per_pair;
    dm::BatchDesc* d_desc = nullptr;
    dm::WorkItem* d_items = nullptr;
    uint32_t* d_words = nullptr;  // acc (2 words per int64) | fix_pairs[n] | bad_tx | next | queue counters
    size_t n_words = 0;
    dm::FixEntry* d_queue = nullptr;
    uint32_t queue_cap = 0;
    void* h_stage = nullptr;
    dm::BatchArgs args{};
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

int build_descs(dm_plan* p, std::vector<dm::BatchDesc>& desc) {
    desc.resize(p->n_inst);
    for (int i = 0; i < p->n_inst; ++i) {
        const dm_instance& in = p->inst[i];
        dm_constellation* c = const_cast<dm_constellation*>(in.c);
        int r = ensure_table8(c);
        if (r) return r;
        dm::BatchDesc& d = desc[i];
        std::memset(&d, 0, sizeof d);
        d.view.table = c->d_table8;
        d.view.row2label = c->d_row2label;
        d.view.tx = in.tx;
        d.view.y = in.y;
        d.view.llr = in.llr;
        d.view.N = in.N;
        d.view.M = c->M;
        d.view.D = c->D;
        d.view.m = c->m;
        d.view.c = exponent_scale(in.sigma2);
        d.view.K = (float)(123 - c->m);
        d.view.flag_thresh = std::ldexp(1.0f, c->m - 102);
        d.view.near_thresh = std::ldexp(1.0f, c->m - 42);
        d.view.want_llr = in.llr ? 1 : 0;
        d.view.tag = i;
        d.kind = p->kind[i];
        d.sub = p->sub[i];
        if (d.kind == dm::kKindMfma) {
            r = ensure_frag(c, p->prec, true);
            if (r) return r;
            d.frag = (const uint4*)c->d_frag8[p->prec];
            d.pv = (const uint16_t*)c->d_pv8[p->prec];
        }
    }
    return DM_OK;
}

// Work list: instances in decreasing order of estimated cost (ns per pair x M x N), each as
// consecutive symbol tiles.  Workgroups claim it in chunks at run time.
void build_work(const dm_plan* p, std::vector<dm::WorkItem>& items) {
    std::vector<int> order(p->n_inst);
    std::vector<double> cost(p->n_inst);
    for (int i = 0; i < p->n_inst; ++i) {
        order[i] = i;
        cost[i] = p->ns_per_pair[i] * p->inst[i].c->M * (double)p->inst[i].N;
    }
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
    for (int i : order) {
        const int64_t tile = (int64_t)dm::batched_tile_symbols(p->kind[i]) * p->sub[i];
        for (int64_t n0 = 0; n0 < p->inst[i].N; n0 += tile) items.push_back(dm::WorkItem{i, 0, n0});
    }
}

int alloc_plan_buffers(dm_plan* p, const std::vector<dm::BatchDesc>& desc, const std::vector<dm::WorkItem>& items) {
    DM_HIP_TRY(hipMalloc(&p->d_desc, desc.size() * sizeof(dm::BatchDesc)));
    DM_HIP_TRY(hipMalloc(&p->d_items, std::max<size_t>(1, items.size()) * sizeof(dm::WorkItem)));
    DM_HIP_TRY(hipMemcpy(p->d_desc, desc.data(), desc.size() * sizeof(dm::BatchDesc), hipMemcpyHostToDevice));
    if (!items.empty())
        DM_HIP_TRY(hipMemcpy(p->d_items, items.data(), items.size() * sizeof(dm::WorkItem), hipMemcpyHostToDevice));
    // the queue's region counters start on a kQueueStride-word boundary after the other words
    const size_t q_off = (((size_t)p->n_inst * dm::kAccSlots * 2 * 2 + p->n_inst + 2 + dm::kQueueStride - 1) /
                          dm::kQueueStride) * dm::kQueueStride;
    p->n_words = q_off + dm::kQueueCounterWords;
    DM_HIP_TRY(hipMalloc(&p->d_words, p->n_words * sizeof(uint32_t)));
    int64_t total_n = 0;
    for (const auto& in : p->inst) total_n += in.N;
    p->queue_cap = (uint32_t)std::min<int64_t>(std::max<int64_t>(total_n, 1024), 1 << 22);
    DM_HIP_TRY(hipMalloc(&p->d_queue, (size_t)p->queue_cap * sizeof(dm::FixEntry)));
    DM_HIP_TRY(hipHostMalloc(&p->h_stage, p->n_words * sizeof(uint32_t), hipHostMallocDefault));
    auto* acc = reinterpret_cast<unsigned long long*>(p->d_words);
    uint32_t* tail = p->d_words + (size_t)p->n_inst * dm::kAccSlots * 2 * 2;
    p->args.desc = p->d_desc;
    p->args.items = p->d_items;
    p->args.n_items = (int32_t)items.size();
    p->args.grab = p->grab;
    p->args.next = tail + p->n_inst + 1;
    p->args.sinks.acc = acc;
    p->args.sinks.fix_pairs = tail;
    p->args.sinks.bad_tx = tail + p->n_inst;
    p->args.sinks.queue_count = p->d_words + q_off;
    p->args.sinks.queue = p->d_queue;
    p->args.sinks.queue_cap = p->queue_cap;
    return DM_OK;
}

int enqueue(dm_plan* p, hipStream_t st) {
    DM_HIP_TRY(dm::launch_zero_words(p->d_words, p->n_words, st));
    DM_HIP_TRY(dm::launch_demap_batched(p->args, p->prec, p->grid, st));
    DM_HIP_TRY(dm::launch_batched_fixup(p->args, p->fix_grid, st));
    return DM_OK;
}

void free_plan(dm_plan* p) {
    if (!p) return;
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
    (void)hipFree(p->d_desc);
    (void)hipFree(p->d_items);
    (void)hipFree(p->d_words);
    (void)hipFree(p->d_queue);
    if (p->h_stage) (void)hipHostFree(p->h_stage);
    delete p;
}

// Plan skeleton without graph: validated instances, kinds, item sizes, per-pair costs and
// claim size set by the caller.
int make_plan(const dm_instance* inst, int n_inst, int prec, const std::vector<int>& kinds,
              const std::vector<int>& subs, const std::vector<double>& cost, int grab, int grid_cap,
              dm_plan** out) {
    auto* p = new (std::nothrow) dm_plan();
    if (!p) return fail(DM_ENOMEM, "host allocation failed");
    p->n_inst = n_inst;
    p->prec = prec;
    p->grab = grab;
    p->inst.assign(inst, inst + n_inst);
    p->kind = kinds;
    p->sub = subs;
    p->ns_per_pair = cost;
    int cus = 0;
    hipError_t e = hipGetDevice(&p->device);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, p->device);
    if (e != hipSuccess) {
        free_plan(p);
        return hip_fail(e, "device query");
    }
    std::vector<dm::BatchDesc> desc;
    std::vector<dm::WorkItem> items;
    int r = build_descs(p, desc);
    if (r) {
        free_plan(p);
        return r;
    }
    p->grid = std::max(1, grid_cap > 0 ? std::min(grid_cap, cus) : cus);
    e = dm::prepare_batched(prec);  // LDS attribute set outside any graph capture
    if (e != hipSuccess) {
        free_plan(p);
        return hip_fail(e, "hipFuncSetAttribute(batched kernel)");
    }
    p->fix_grid = cus * 4;
    build_work(p, items);
    r = alloc_plan_buffers(p, desc, items);
    if (r) {
        free_plan(p);
        return r;
    }
    *out = p;
    return DM_OK;
}

int validate_instances(const dm_instance* inst, int n_inst, int prec) {
    if (!inst || n_inst < 1) return fail(DM_EINVAL, "need at least one instance");
    if (prec < DM_PREC_FP32 || prec > DM_PREC_FP16X3) return fail(DM_EINVAL, "unknown precision %d", prec);
    int dev = -1;
    DM_HIP_TRY(hipGetDevice(&dev));
    for (int i = 0; i < n_inst; ++i) {
        const dm_instance& in = inst[i];
        if (!in.c) return fail(DM_EINVAL, "instance %d has no constellation", i);
        if (in.c->device != dev) return fail(DM_EINVAL, "instance %d lives on another device", i);
        if (in.c->D > 8) return fail(DM_EUNSUPPORTED, "batched plans support D <= 8 (instance %d has D=%d)", i, in.c->D);
        if ((size_t)std::max(16, in.c->M) * 8 * 4 > (size_t)dm::kBatchedLdsBytes)
            return fail(DM_EUNSUPPORTED, "instance %d: M=%d exceeds the batched table size", i, in.c->M);
        if (in.N < 0 || in.N >= (int64_t(1) << 31)) return fail(DM_EINVAL, "instance %d: bad N", i);
        int r = validate_sigma2(in.sigma2);
        if (r) return r;
        if (in.N > 0) {
            if ((r = check_device_ptr(in.y, "instance y", dev))) return r;
            if (in.tx && (r = check_device_ptr(in.tx, "instance tx", dev))) return r;
            if (in.llr && (r = check_device_ptr(in.llr, "instance llr", dev))) return r;
        }
        if ((prec == DM_PREC_FP16 || prec == DM_PREC_FP16X3) && mfma_possible(in.c, prec) &&
            (in.c->max_norm >= 60000.0f || exponent_scale(in.sigma2) >= 30000.0f))
            return fail(DM_EUNSUPPORTED, "instance %d is outside the FP16 operand range", i);
    }
    return DM_OK;
}

// Best time (ms) of two launches after one warm-up launch of a plan on a private stream.
int time_plan(dm_plan* p, float* best_ms) {
    hipStream_t st = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    float best = 1e30f;
    int r = DM_OK;
    for (int rep = 0; e == hipSuccess && rep < 3; ++rep) {
        (void)hipEventRecord(e0, st);
        if ((r = enqueue(p, st))) break;
        (void)hipEventRecord(e1, st);
        e = hipEventSynchronize(e1);
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (rep > 0) best = std::min(best, ms);  // the first launch warms up
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (st) (void)hipStreamDestroy(st);
    if (r) return r;
    if (e != hipSuccess) return hip_fail(e, "autotune timing");
    *best_ms = best;
    return DM_OK;
}

// Time one class with one shape (kind, item size) on a probe block of about kProbeItemsPerCu
// work items per CU: copies of the instance's first symbols (read only, no LLRs written).
int time_candidate(const dm_instance& in, int prec, int kind, int sub, int cus, double* ns_per_pair) {
    const int64_t want = (int64_t)kProbeItemsPerCu * cus * dm::batched_tile_symbols(kind) * sub;
    dm_instance probe = in;
    probe.N = std::min<int64_t>(in.N, want);
    probe.llr = nullptr;
    const int copies = (int)std::min<int64_t>(kProbeCopies, (want + probe.N - 1) / std::max<int64_t>(probe.N, 1));
    std::vector<dm_instance> insts(copies, probe);
    dm_plan* p = nullptr;
    int r = make_plan(insts.data(), copies, prec, std::vector<int>(copies, kind), std::vector<int>(copies, sub),
                      std::vector<double>(copies, 1.0), kGrabDefault, 0, &p);
    if (r) return r;
    float ms = 0.0f;
    r = time_plan(p, &ms);
    free_plan(p);
    if (r) return r;
    *ns_per_pair = (double)ms * 1e6 / ((double)std::max<int64_t>(probe.N, 1) * copies * in.c->M);
    return DM_OK;
}

}  // namespace

extern "C" {

int dm_plan_create(const dm_instance* inst, int n_inst, int prec, int flags, dm_plan** out) {
    if (!out) return fail(DM_EINVAL, "null plan pointer");
    *out = nullptr;
    int r = validate_instances(inst, n_inst, prec);
    if (r) return r;
    const int force_items = (flags >> 8) & 0xF, force_claim = (flags >> 12) & 0xF;
    if (force_items > 3) return fail(DM_EINVAL, "DM_PLAN_ITEMS(k) needs k in 1..3");
    if (force_claim > 4) return fail(DM_EINVAL, "DM_PLAN_CLAIM(k) needs k in 1..4");
    int cus = 0, dev = 0;
    DM_HIP_TRY(hipGetDevice(&dev));
    DM_HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    std::vector<int> kinds(n_inst), subs(n_inst, force_items ? 1 << (force_items - 1) : 1);
    std::vector<double> cost(n_inst, 0.0);
    for (int i = 0; i < n_inst; ++i) {
        const dm_constellation* c = inst[i].c;
        const bool can_mfma = mfma_possible(c, prec);
        if (flags & DM_PLAN_FORCE_VALU) {
            kinds[i] = dm::kKindValu;
        } else if (flags & DM_PLAN_FORCE_MFMA) {
            if (!can_mfma) return fail(DM_EUNSUPPORTED, "instance %d cannot use the MFMA body", i);
            kinds[i] = dm::kKindMfma;
        } else {
            kinds[i] = can_mfma ? dm::kKindMfma : dm::kKindValu;
        }
        // Default cost model: measured-order-of-magnitude ns per pair of each body.
        cost[i] = kinds[i] == dm::kKindMfma ? 1.6e-4 : 5.0e-4;
    }
    const bool tune = (flags & DM_PLAN_AUTOTUNE) != 0;
    if (tune) {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        load_tune_cache();
        bool tuned = false;
        for (int i = 0; i < n_inst; ++i) {
            const dm_constellation* c = inst[i].c;
            if (inst[i].N == 0) continue;
            double best = 0.0;
            int best_kind = kinds[i], best_sub = subs[i];
            for (int kind = dm::kKindValu; kind <= dm::kKindMfma; ++kind) {
                if (kind == dm::kKindMfma && !mfma_possible(c, prec)) continue;
                if ((flags & DM_PLAN_FORCE_VALU) && kind != dm::kKindValu) continue;
                if ((flags & DM_PLAN_FORCE_MFMA) && kind != dm::kKindMfma) continue;
                for (int sub : kSubs) {
                    if (force_items && sub != subs[i]) continue;
                    const TuneKey key{c->M, c->D, prec, kind, sub};
                    auto it = g_tune.find(key);
                    double ns;
                    if (it != g_tune.end()) {
                        ns = it->second;
                    } else {
                        r = time_candidate(inst[i], prec, kind, sub, cus, &ns);
                        if (r) return r;
                        g_tune[key] = ns;
                        tuned = true;
                    }
                    if (best == 0.0 || ns < best) {
                        best = ns;
                        best_kind = kind;
                        best_sub = sub;
                    }
                }
            }
            kinds[i] = best_kind;
            subs[i] = best_sub;
            cost[i] = best;
        }
        if (tuned) save_tune_cache();
    }
    // Claim size: forced, the default, or the fastest whole plan (timed without LLR writes).
    int grab = force_claim ? 1 << (force_claim - 1) : kGrabDefault;
    if (tune && !force_claim) {
        std::vector<dm_instance> quiet(inst, inst + n_inst);
        for (auto& q : quiet) q.llr = nullptr;
        float best_ms = 0.0f;
        for (int g : kGrabs) {
            dm_plan* tp = nullptr;
            if ((r = make_plan(quiet.data(), n_inst, prec, kinds, subs, cost, g, 0, &tp))) return r;
            float ms = 0.0f;
            r = time_plan(tp, &ms);
            free_plan(tp);
            if (r) return r;
            if (best_ms == 0.0f || ms < best_ms) {
                best_ms = ms;
                grab = g;
            }
        }
    }
    dm_plan* p = nullptr;
    r = make_plan(inst, n_inst, prec, kinds, subs, cost, grab, 0, &p);
    if (r) return r;
    // Capture zero-fill + batched kernel + fix-up into a graph on a private stream.
    hipError_t e = hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        r = enqueue(p, p->cap_stream);
        hipGraph_t g = nullptr;
        const hipError_t e2 = hipStreamEndCapture(p->cap_stream, &g);
        p->graph = g;
        if (!r && e2 != hipSuccess) e = e2;
    }
    if (e == hipSuccess && !r) e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
    if (r || e != hipSuccess) {
        free_plan(p);
        return r ? r : hip_fail(e, "graph capture");
    }
    *out = p;
    return DM_OK;
}

int dm_plan_launch(dm_plan* p, void* stream) {
    if (!p) return fail(DM_EINVAL, "null plan");
    DM_HIP_TRY(hipGraphLaunch(p->exec, (hipStream_t)stream));
    return DM_OK;
}

int dm_plan_results(dm_plan* p, double* gmi, double* mi, int64_t* fixup_pairs, void* stream) {
    if (!p || !gmi) return fail(DM_EINVAL, "null argument");
    hipStream_t st = (hipStream_t)stream;
    DM_HIP_TRY(hipMemcpyAsync(p->h_stage, p->d_words, p->n_words * sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    DM_HIP_TRY(hipStreamSynchronize(st));
    const auto* acc = reinterpret_cast<const unsigned long long*>(p->h_stage);
    const auto* tail = reinterpret_cast<const uint32_t*>(p->h_stage) + (size_t)p->n_inst * dm::kAccSlots * 2 * 2;
    if (tail[p->n_inst]) return fail(DM_EINVAL, "a transmitted index is >= M");
    for (int i = 0; i < p->n_inst; ++i) {
        long long gs = 0, ms = 0;
        for (int k = 0; k < dm::kAccSlots; ++k) {
            gs += (long long)acc[((size_t)i * dm::kAccSlots + k) * 2 + 0];
            ms += (long long)acc[((size_t)i * dm::kAccSlots + k) * 2 + 1];
        }
        const double N = (double)p->inst[i].N;
        const bool has = p->inst[i].tx && p->inst[i].N > 0;
        gmi[i] = has ? (double)gs / dm::kFixScale / N : NAN;
        if (mi) mi[i] = has ? (double)ms / dm::kFixScale / N : NAN;
        if (fixup_pairs) fixup_pairs[i] = tail[i];
    }
    return DM_OK;
}

int dm_plan_info(const dm_plan* p, int* kinds, double* ns_per_pair, int32_t* item_symbols) {
    if (!p) return fail(DM_EINVAL, "null plan");
    for (int i = 0; i < p->n_inst; ++i) {
        if (kinds) kinds[i] = p->kind[i];
        if (ns_per_pair) ns_per_pair[i] = p->ns_per_pair[i];
        if (item_symbols) item_symbols[i] = dm::batched_tile_symbols(p->kind[i]) * p->sub[i];
    }
    return DM_OK;
}

int dm_plan_stats(const dm_plan* p, int64_t* n_items, int32_t* claim_items, int32_t* grid) {
    if (!p) return fail(DM_EINVAL, "null plan");
    if (n_items) *n_items = p->args.n_items;
    if (claim_items) *claim_items = p->args.grab;
    if (grid) *grid = p->grid;
    return DM_OK;
}

void dm_plan_destroy(dm_plan* p) { free_plan(p); }

int dm_demap_batched(const dm_instance* inst, int n_inst, int prec, int flags, double* gmi, double* mi,
                     void* stream) {
    dm_plan* p = nullptr;
    int r = dm_plan_create(inst, n_inst, prec, flags, &p);
    if (r) return r;
    r = dm_plan_launch(p, stream);
    if (!r) r = dm_plan_results(p, gmi, mi, nullptr, stream);
    dm_plan_destroy(p);
    return r;
}

}  // extern "C"
