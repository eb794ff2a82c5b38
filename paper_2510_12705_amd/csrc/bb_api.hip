// bb_api.hip -- host side of the C ABI declared in include/bb.h.
//
// Planning (stages of Algorithm 1, per-stage half-step lag), argument checks,
// stream-ordered working memory, and the launch sequence
//   fill(counters) -> pack -> stage kernel per bandwidth-reduction stage -> extract.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <vector>

#include "bb.h"
#include "bb_internal.h"
#include "bb_plan.h"

namespace {

constexpr int kMaxXcd = 16;  // per-XCD claim counters kept per stage

// The device's error word (watchdog): written by kernels, read and cleared by
// bb_stream_status.  A device global, so that setting up a device allocates nothing.
__device__ int g_err_word;

}  // namespace

// Working memory of bb_reduce_noalloc: one call's working band and dependency
// counters, in a static device array that every device holding the library keeps
// until the process ends.  Host code never passes this name to a kernel or a
// copy: it is a host-side stand-in for the symbol, and device_state() resolves
// each device's own address of it with hipGetSymbolAddress.
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

struct DeviceState {
    bool init = false;
    int cus = 0;
    size_t lds_per_block = 65536;  // largest dynamic LDS allocation of one workgroup
    int nxcd = 1;                  // XCDs (accelerator complex dies), each with its own L2
    int* err_dev = nullptr;        // this device's copy of g_err_word
    char* scratch_dev = nullptr;   // this device's copy of `scratch` (bb_reduce_noalloc)
    hipStream_t aux = nullptr;     // second stream of bb_reduce_vectors (default priority)
};

std::mutex g_mu;
bb_params_t g_params = {0, 0, 0, 0, 0, 0};
std::vector<DeviceState> g_dev;

struct Timing {
    bool on = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> events;
};
Timing g_timing;

unsigned spin_limit() {
    static unsigned v = [] {
        const char* s = getenv("BB_SPIN_LIMIT");
        long x = s ? strtol(s, nullptr, 10) : 0;
        return x > 0 ? (unsigned)x : (1u << 22);
    }();
    return v;
}

int device_state(DeviceState** out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return BB_ERR_NODEVICE;
    std::lock_guard<std::mutex> lk(g_mu);
    if ((int)g_dev.size() <= dev) g_dev.resize(dev + 1);
    DeviceState& s = g_dev[dev];
    if (!s.init) {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return BB_ERR_NODEVICE;
        s.cus = prop.multiProcessorCount;
        if (prop.sharedMemPerBlock > 0) s.lds_per_block = prop.sharedMemPerBlock;
        int nx = 1;
        if (hipDeviceGetAttribute(&nx, hipDeviceAttributeNumberOfXccs, dev) == hipSuccess && nx >= 1)
            s.nxcd = std::min(nx, (int)kMaxXcd);
        if (hipGetSymbolAddress((void**)&s.err_dev, HIP_SYMBOL(g_err_word)) != hipSuccess) return BB_ERR_HIP;
        if (hipGetSymbolAddress((void**)&s.scratch_dev, HIP_SYMBOL(scratch)) != hipSuccess) return BB_ERR_HIP;
        hipMemPool_t pool;
        if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
            uint64_t thr = UINT64_MAX;  // keep freed working memory cached in the pool
            hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
        }
        s.init = true;
    }
    *out = &s;
    return BB_OK;
}

size_t elem_size(int dtype) { return dtype == BB_F64 ? 8 : dtype == BB_F32 ? 4 : 2; }
size_t elem_size_c(int dtype) { return dtype == BB_F64 ? 8 : 4; }  // compute type held in LDS

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Launch shape.  ntl / lanes are those of the first stage; unless fixed by the
// caller (or an autotuned entry) they are re-derived for every stage from its
// window height (stage_shape).
struct Launch {
    int tw, ntl, lanes, groups_per_cu, lag, xcd_run;
    bool ntl_fixed, lanes_fixed;
    size_t lds_limit;
};

bb_params_t current_params() {
    std::lock_guard<std::mutex> lk(g_mu);
    return g_params;
}

// Effective launch shape: a nonzero field of `p` wins, then a nonzero field of an
// autotuned entry for this shape (if use_cache), then the built-in default.
// Workgroups per CU default to 2 for one band (more only lengthen each sweep's
// half-steps) and to 4 for a batch, whose many independent sweeps fill every
// workgroup the CU can hold (measured: 512 ragged FP32 bands 647 ms -> 392 ms).
Launch resolve(int64_t n, int64_t b, int dtype, size_t lds_limit, bb_params_t p, bool use_cache = true,
               int default_groups_per_cu = 2) {
    bbp::Tuned t;
    if (use_cache && bbp::autotune_lookup(n, b, dtype, &t)) {
        if (!p.tw) p.tw = t.p.tw;
        if (!p.threads_per_window) p.threads_per_window = t.p.threads_per_window;
        if (!p.sweeps_per_group) p.sweeps_per_group = t.p.sweeps_per_group;
        if (!p.groups_per_cu) p.groups_per_cu = t.p.groups_per_cu;
        if (!p.lag) p.lag = t.p.lag;
        if (!p.xcd_run) p.xcd_run = t.p.xcd_run;
    }
    Launch L;
    L.tw = p.tw ? p.tw : bbp::default_tw(dtype);
    int rows = (int)std::min<int64_t>(b, std::max<int64_t>(n - 1, 1)) + L.tw;
    L.ntl = p.threads_per_window ? p.threads_per_window : bbp::default_threads(rows, dtype);
    L.lanes = p.sweeps_per_group ? p.sweeps_per_group : bbp::default_lanes(L.ntl, dtype);
    L.ntl_fixed = p.threads_per_window != 0;
    L.lanes_fixed = p.sweeps_per_group != 0;
    L.lds_limit = lds_limit;
    L.groups_per_cu = p.groups_per_cu ? p.groups_per_cu : default_groups_per_cu;
    L.lag = p.lag;
    L.xcd_run = p.xcd_run ? p.xcd_run : 2;
    // fit the workgroup's LDS (corners + staging blocks) and thread limits; a
    // 64-wide tile writes 65-entry segments, one thread per entry
    const int twm = bbp::kernel_twm(L.tw);
    if (twm > 32 && L.ntl < 128) L.ntl = 128;
    while (L.lanes > 1 && bbk::stage_lds_bytes(dtype, twm, L.ntl, L.lanes) > lds_limit) --L.lanes;
    while (L.lanes > 1 && L.lanes * L.ntl > bbk::stage_max_threads(twm)) --L.lanes;
    return L;
}

// threads per window and sweeps per workgroup for one stage
void stage_shape(const Launch& L, const bbp::Stage& sg, int dtype, int* ntl, int* lanes) {
    const int twm = bbp::kernel_twm(sg.tw);
    int nt = L.ntl_fixed ? L.ntl : bbp::default_threads(sg.b + sg.tw, dtype);
    if (twm > 32 && nt < 128) nt = 128;
    int ln = L.lanes_fixed ? L.lanes : bbp::default_lanes(nt, dtype);
    while (ln > 1 && bbk::stage_lds_bytes(dtype, twm, nt, ln) > L.lds_limit) --ln;
    while (ln > 1 && ln * nt > bbk::stage_max_threads(twm)) --ln;
    *ntl = nt;
    *lanes = ln;
}

struct Workspace {
    size_t band_bytes = 0, counter_bytes = 0, total = 0;
    int64_t ldw = 0, uo = 0, max_sweeps = 0;
    int nstages = 0;
    // counter words: progress[nstages][max_sweeps] | per stage kMaxXcd claim words and
    // an abort word | FP16 amax per stage | FP16 exps[nstages + 1]; all zero-initialised
    // per call
    int64_t off_claim = 0, off_amax = 0, off_exps = 0, ncounters = 0;
};

Workspace workspace_layout(int64_t n, int64_t b, int dtype, int tw) {
    Workspace w;
    const int tw0 = b > 1 ? bbp::stage_first(b, tw).tw : 0;
    w.uo = std::max<int64_t>(b + tw0, 1);
    w.ldw = align_up((size_t)(w.uo + tw0 + 1), 2);
    w.nstages = bbp::stage_count(b, tw);
    w.max_sweeps = std::max<int64_t>(n, 1);
    w.band_bytes = align_up((size_t)(n * w.ldw) * elem_size(dtype), 256);
    w.off_claim = w.nstages * w.max_sweeps;
    w.off_amax = w.off_claim + (kMaxXcd + 1) * w.nstages;
    w.off_exps = w.off_amax + w.nstages;
    w.ncounters = w.off_exps + w.nstages + 1;
    w.counter_bytes = align_up(sizeof(int) * (size_t)w.ncounters, 256);
    w.total = w.band_bytes + w.counter_bytes;
    return w;
}

int check_hip(hipError_t e) { return e == hipSuccess ? BB_OK : BB_ERR_HIP; }

// Read (and with `clear`, reset) the device's error word; the caller has synchronised.
int read_err_word(DeviceState* ds, bool clear) {
    int v = 0;
    if (hipMemcpy(&v, ds->err_dev, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess) return BB_ERR_HIP;
    if (v && clear) {
        const int z = 0;
        if (hipMemcpy(ds->err_dev, &z, sizeof(int), hipMemcpyHostToDevice) != hipSuccess) return BB_ERR_HIP;
    }
    return v;
}

// The stage kernels address a window with 32-bit byte offsets from a wave-uniform
// base; the largest spans kWave + TW + 2 band columns.  True when they fit.
bool window_offsets_fit(const Workspace& w, int dtype) {
    return (int64_t)(64 + bbp::kMaxTW + 2) * w.ldw * (int64_t)elem_size(dtype) < ((int64_t)1 << 32);
}

// ---------------------------------------------------------------------------
// Ragged batch plan, cached per (shapes, dtype, launch parameters, stream): the
// device workspace is allocated once with hipMalloc and reused, so repeated
// calls allocate nothing and can be captured into a hipGraph.  Calls that share
// a plan must not overlap in time (they share its workspace); calls on
// different streams get different plans.
// ---------------------------------------------------------------------------
struct BatchPlan {
    uint64_t key = 0;  // hash of the fields below: a pre-filter only, matched exactly after it
    hipStream_t stream = nullptr;
    int count = 0, dtype = 0, tw = 0, ntl = 0, lanes = 0, twm = 0, lag = 0;
    std::vector<int64_t> ns, bs;  // the caller's n[] and b[]
    int64_t max_elems = 0, max_n = 0;
    int ntasks = 0, nprogress = 0, nexps = 0;
    std::vector<bbk::BatchMatrix> mats;
    std::vector<bbk::BatchStage> stages;
    std::vector<bbk::BatchTask> tasks;
    char* dev = nullptr;   // device workspace
    size_t dev_bytes = 0;
    size_t off_counters = 0, off_mats = 0, off_stages = 0, off_tasks = 0, off_ptrs = 0;
    int64_t ncounters = 0;
    void* pinned = nullptr;          // staging for the pointer arrays of direct (uncaptured) calls
    void* pinned_capture = nullptr;  // staging read by captured copies when a graph is replayed
    hipEvent_t staged = nullptr;
    bool staged_pending = false;

    bool matches(int64_t cnt, const int64_t* n, const int64_t* b, int dt, const Launch& L, hipStream_t st) const {
        if (stream != st || count != cnt || dtype != dt || tw != L.tw || ntl != L.ntl || lanes != L.lanes ||
            lag != L.lag)
            return false;
        for (int64_t i = 0; i < cnt; ++i)
            if (ns[(size_t)i] != n[i] || bs[(size_t)i] != b[i]) return false;
        return true;
    }
};

std::vector<BatchPlan*> g_batch_plans;

// Tuned parameters of the batched form, keyed on the exact batch (dtype, n[], b[]).
struct BatchTuned {
    int dtype;
    std::vector<int64_t> ns, bs;
    bb_params_t p;
};
std::vector<BatchTuned> g_batch_tuned;

bool batch_tuned_lookup(int64_t count, const int64_t* n, const int64_t* b, int dtype, bb_params_t* p) {
    std::lock_guard<std::mutex> lk(g_mu);
    for (const BatchTuned& t : g_batch_tuned) {
        if (t.dtype != dtype || (int64_t)t.ns.size() != count) continue;
        if (std::equal(t.ns.begin(), t.ns.end(), n) && std::equal(t.bs.begin(), t.bs.end(), b)) {
            *p = t.p;
            return true;
        }
    }
    return false;
}

void batch_tuned_store(int64_t count, const int64_t* n, const int64_t* b, int dtype, const bb_params_t& p) {
    std::lock_guard<std::mutex> lk(g_mu);
    for (BatchTuned& t : g_batch_tuned)
        if (t.dtype == dtype && (int64_t)t.ns.size() == count && std::equal(t.ns.begin(), t.ns.end(), n) &&
            std::equal(t.bs.begin(), t.bs.end(), b)) {
            t.p = p;
            return;
        }
    g_batch_tuned.push_back(BatchTuned{dtype, std::vector<int64_t>(n, n + count), std::vector<int64_t>(b, b + count), p});
}



uint64_t mix(uint64_t h, uint64_t v) {
    h ^= v + 0x9E3779B97F4A7C15ull + (h << 6) + (h >> 2);
    return h;
}

int batch_plan(int64_t count, const int64_t* n, const int64_t* b, int dtype, const Launch& L, hipStream_t st,
               BatchPlan** out) {
    uint64_t key = mix(mix(mix(mix(mix(mix(0, (uint64_t)count), (uint64_t)dtype), (uint64_t)L.tw), (uint64_t)L.ntl),
                           (uint64_t)L.lanes),
                       (uint64_t)L.lag);
    for (int64_t i = 0; i < count; ++i) key = mix(mix(key, (uint64_t)n[i]), (uint64_t)b[i]);
    {
        std::lock_guard<std::mutex> lk(g_mu);
        for (BatchPlan* p : g_batch_plans)
            if (p->key == key && p->matches(count, n, b, dtype, L, st)) {
                *out = p;
                return BB_OK;
            }
    }
    for (int64_t i = 0; i < count; ++i) {
        const int64_t bb = n[i] > 0 ? std::min<int64_t>(b[i], n[i] - 1) : 0;
        if (!window_offsets_fit(workspace_layout(std::max<int64_t>(n[i], 1), bb, dtype, L.tw), dtype))
            return BB_ERR_UNSUPPORTED;
    }
    BatchPlan* P = new BatchPlan();
    P->key = key;
    P->stream = st;
    P->count = (int)count;
    P->dtype = dtype;
    P->tw = L.tw;
    P->ntl = L.ntl;
    P->lanes = L.lanes;
    P->lag = L.lag;
    P->ns.assign(n, n + count);
    P->bs.assign(b, b + count);
    P->twm = bbp::kernel_twm(L.tw);
    size_t band_off = 0;
    std::vector<size_t> band_offs((size_t)count);
    int max_stages = 0;
    for (int64_t i = 0; i < count; ++i) {
        bbk::BatchMatrix M{};
        const int64_t bb = n[i] > 0 ? std::min<int64_t>(b[i], n[i] - 1) : 0;
        Workspace w = workspace_layout(std::max<int64_t>(n[i], 1), bb, dtype, L.tw);
        bbp::Plan pl = bbp::make_plan(bb, L.tw);
        M.S = w.ldw - 1;
        M.uo = w.uo;
        M.n = (int)n[i];
        M.b = (int)bb;
        M.b_in = (int)b[i];
        M.nstages = (int)pl.stages.size();
        M.stage_off = (int)P->stages.size();
        M.exp_off = P->nexps;
        P->nexps += M.nstages + 1;
        band_offs[(size_t)i] = band_off;
        band_off += w.band_bytes;
        P->max_elems = std::max<int64_t>(P->max_elems, (int64_t)n[i] * w.ldw);
        P->max_n = std::max<int64_t>(P->max_n, n[i]);
        for (const bbp::Stage& sg : pl.stages) {
            bbk::BatchStage S{};
            S.b = sg.b;
            S.tw = sg.tw;
            S.c = sg.c;
            S.H = std::max(sg.lag, L.lag);
            S.nsweeps = (int)std::max<int64_t>(n[i] - sg.c - 1, 0);
            S.ngroups = (S.nsweeps + L.lanes - 1) / L.lanes;
            S.prog_off = P->nprogress;
            P->nprogress += S.ngroups;
            P->stages.push_back(S);
        }
        max_stages = std::max(max_stages, M.nstages);
        P->mats.push_back(M);
    }
    // tasks ordered by (stage, group, matrix): every dependency precedes its task
    for (int sidx = 0; sidx < max_stages; ++sidx) {
        int max_groups = 0;
        for (const auto& M : P->mats)
            if (sidx < M.nstages) max_groups = std::max(max_groups, P->stages[M.stage_off + sidx].ngroups);
        for (int q = 0; q < max_groups; ++q)
            for (int i = 0; i < P->count; ++i) {
                const auto& M = P->mats[i];
                if (sidx < M.nstages && q < P->stages[M.stage_off + sidx].ngroups)
                    P->tasks.push_back(bbk::BatchTask{i, sidx, q});
            }
    }
    P->ntasks = (int)P->tasks.size();
    // device layout: bands | counters (progress, exps, claim, abort) | mats | stages | tasks | pointer arrays
    P->ncounters = (int64_t)P->nprogress + P->nexps + 2;
    P->off_counters = align_up(band_off, 256);
    P->off_mats = align_up(P->off_counters + sizeof(int) * (size_t)P->ncounters, 256);
    P->off_stages = align_up(P->off_mats + sizeof(bbk::BatchMatrix) * P->mats.size(), 256);
    P->off_tasks = align_up(P->off_stages + sizeof(bbk::BatchStage) * std::max<size_t>(P->stages.size(), 1), 256);
    P->off_ptrs = align_up(P->off_tasks + sizeof(bbk::BatchTask) * std::max<size_t>(P->tasks.size(), 1), 256);
    P->dev_bytes = P->off_ptrs + 4 * sizeof(void*) * (size_t)count;
    if (hipMalloc((void**)&P->dev, P->dev_bytes) != hipSuccess) {
        delete P;
        return BB_ERR_NOMEM;
    }
    for (int64_t i = 0; i < count; ++i) P->mats[(size_t)i].W = P->dev + band_offs[(size_t)i];
    if (hipHostMalloc(&P->pinned, 4 * sizeof(void*) * (size_t)count, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc(&P->pinned_capture, 4 * sizeof(void*) * (size_t)count, hipHostMallocDefault) != hipSuccess ||
        hipEventCreateWithFlags(&P->staged, hipEventDisableTiming) != hipSuccess) {
        if (P->pinned) (void)hipHostFree(P->pinned);
        if (P->pinned_capture) (void)hipHostFree(P->pinned_capture);
        (void)hipFree(P->dev);
        delete P;
        return BB_ERR_NOMEM;
    }
    // static metadata: one synchronous upload when the plan is built
    if (hipMemcpy(P->dev + P->off_mats, P->mats.data(), sizeof(bbk::BatchMatrix) * P->mats.size(),
                  hipMemcpyHostToDevice) != hipSuccess ||
        (!P->stages.empty() && hipMemcpy(P->dev + P->off_stages, P->stages.data(),
                                         sizeof(bbk::BatchStage) * P->stages.size(), hipMemcpyHostToDevice) != hipSuccess) ||
        (!P->tasks.empty() && hipMemcpy(P->dev + P->off_tasks, P->tasks.data(), sizeof(bbk::BatchTask) * P->tasks.size(),
                                        hipMemcpyHostToDevice) != hipSuccess)) {
        (void)hipFree(P->dev);
        delete P;
        return BB_ERR_HIP;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    g_batch_plans.push_back(P);
    *out = P;
    return BB_OK;
}

int batch_run(BatchPlan* P, DeviceState* ds, const void* const* band, const int64_t* ldband, double* const* d,
              double* const* e, const Launch& L, hipStream_t st) {
    const size_t cnt = (size_t)P->count;
    // Direct calls stage the pointer arrays in `pinned`, which may still feed the
    // previous direct call's copy (hence the event wait).  A call captured into a
    // graph executes nothing now: its copy reads `pinned_capture` whenever the graph
    // is replayed, so direct calls never overwrite what a queued replay reads, and
    // a capture never overwrites what a queued direct copy reads.  Replays use the
    // pointers of the most recent capture with this plan.
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) != hipSuccess) return BB_ERR_HIP;
    const bool capturing = cs != hipStreamCaptureStatusNone;
    if (!capturing && P->staged_pending && hipEventSynchronize(P->staged) != hipSuccess) return BB_ERR_HIP;
    void** host = static_cast<void**>(capturing ? P->pinned_capture : P->pinned);
    for (size_t i = 0; i < cnt; ++i) {
        host[i] = const_cast<void*>(band[i]);
        host[cnt + i] = reinterpret_cast<void*>(ldband[i]);
        host[2 * cnt + i] = d[i];
        host[3 * cnt + i] = e[i];
    }
    char* ptrs = P->dev + P->off_ptrs;
    int rc = check_hip(hipMemcpyAsync(ptrs, host, 4 * sizeof(void*) * cnt, hipMemcpyHostToDevice, st));
    if (!rc && !capturing) {
        rc = check_hip(hipEventRecord(P->staged, st));
        P->staged_pending = rc == BB_OK;
    }
    int* counters = reinterpret_cast<int*>(P->dev + P->off_counters);
    const auto* mats = reinterpret_cast<const bbk::BatchMatrix*>(P->dev + P->off_mats);
    if (!rc) rc = check_hip(bbk::launch_fill(counters, P->ncounters, 0, st));
    if (!rc)
        rc = check_hip(bbk::launch_pack_batched(P->dtype, mats, P->count, P->max_elems,
                                                reinterpret_cast<const void* const*>(ptrs),
                                                reinterpret_cast<const int64_t*>(ptrs + sizeof(void*) * cnt), st));
    if (!rc && P->ntasks > 0) {
        bbk::BatchArgs a;
        a.mats = mats;
        a.stages = reinterpret_cast<const bbk::BatchStage*>(P->dev + P->off_stages);
        a.tasks = reinterpret_cast<const bbk::BatchTask*>(P->dev + P->off_tasks);
        a.ntasks = P->ntasks;
        a.progress = counters;
        a.exps = counters + P->nprogress;
        a.claim = counters + P->nprogress + P->nexps;
        a.abort_flag = a.claim + 1;
        a.err_word = ds->err_dev;
        a.spin_limit = spin_limit();
        const int grid = (int)std::min<int64_t>(P->ntasks, (int64_t)ds->cus * L.groups_per_cu);
        rc = check_hip(bbk::launch_batched(P->dtype, a, P->twm, P->ntl, P->lanes, grid, st));
    }
    if (!rc)
        rc = check_hip(bbk::launch_extract_batched(P->dtype, mats, P->count, P->max_n,
                                                   P->dtype == BB_F16 ? counters + P->nprogress : nullptr,
                                                   reinterpret_cast<double* const*>(ptrs + 2 * sizeof(void*) * cnt),
                                                   reinterpret_cast<double* const*>(ptrs + 3 * sizeof(void*) * cnt), st));
    return rc;
}

void batch_plans_clear() {
    std::lock_guard<std::mutex> lk(g_mu);
    for (BatchPlan* p : g_batch_plans) {
        if (p->staged_pending) (void)hipEventSynchronize(p->staged);
        (void)hipEventDestroy(p->staged);
        (void)hipHostFree(p->pinned);
        (void)hipHostFree(p->pinned_capture);
        (void)hipFree(p->dev);
        delete p;
    }
    g_batch_plans.clear();
}

}  // namespace

extern "C" {

static int reduce_impl(int64_t n, int64_t b, int dtype, const void* band, int64_t ldband, double* d, double* e,
                       hipStream_t st, DeviceState* ds, const bb_params_t& params, bool use_cache);

int bb_reduce(int64_t n, int64_t b, bb_dtype_t dtype, const void* band, int64_t ldband, double* d, double* e,
              void* stream) {
    if (n < 0) return -1;
    if (b < 0) return -2;
    if (dtype != BB_F64 && dtype != BB_F32 && dtype != BB_F16) return -3;
    if (n > 0 && !band) return -4;
    if (ldband < b + 1) return -5;
    if (n > 0 && !d) return -6;
    if (n > 1 && !e) return -7;
    if (n > (int64_t)1 << 30) return -1;
    if (n == 0) return BB_OK;
    DeviceState* ds = nullptr;
    int rc = device_state(&ds);
    if (rc) return rc;
    return reduce_impl(n, b, dtype, band, ldband, d, e, (hipStream_t)stream, ds, current_params(), true);
}

// A validated bb_reduce call: launch shape and working-memory layout.
struct Call {
    int64_t n = 0, b_in = 0, bb = 0;  // order, caller's bandwidth, bandwidth clamped to n - 1
    int dtype = 0;
    Launch L{};
    Workspace ws{};
};

static int prepare_call(int64_t n, int64_t b, int dtype, DeviceState* ds, const bb_params_t& params, bool use_cache,
                        Call* c) {
    c->n = n;
    c->b_in = b;
    c->bb = std::min<int64_t>(b, n - 1);
    c->dtype = dtype;
    c->L = resolve(n, c->bb, dtype, ds->lds_per_block, params, use_cache);
    if (c->L.tw < 1 || c->L.tw > bbp::max_tw(dtype)) return BB_ERR_UNSUPPORTED;
    c->ws = workspace_layout(n, c->bb, dtype, c->L.tw);
    if (!window_offsets_fit(c->ws, dtype)) return BB_ERR_UNSUPPORTED;
    return BB_OK;
}

// Reflector log of a call that forms the singular vectors: per stage, right-task
// slots [step j][sweep r] then left-task slots, wlog doubles each (tau, v_1..v_TW).
struct VecLog {
    double* base = nullptr;
    int wlog = 0;
    std::vector<int64_t> off;     // per stage: offset of its slots (doubles)
    std::vector<int> nsteps;      // per stage: steps of its longest sweep (sweep 0)
    int64_t doubles = 0;          // total size
    std::vector<hipEvent_t> stage_done;  // if set: recorded on the call's stream after stage s
};

static VecLog veclog_layout(int64_t n, int64_t bb, int tw) {
    VecLog v;
    if (bb <= 1) return v;
    v.wlog = bbp::stage_first(bb, tw).tw + 1;
    for (bbp::Stage sg = bbp::stage_first(bb, tw);; sg = bbp::stage_next(sg, tw)) {
        const int64_t nsw = std::max<int64_t>(n - sg.c - 1, 0);
        const int nst = nsw > 0 ? (int)(1 + (n - 2 - sg.c) / sg.b) : 0;
        v.off.push_back(v.doubles);
        v.nsteps.push_back(nst);
        v.doubles += 2 * (int64_t)nst * nsw * v.wlog;
        if (sg.c <= 1) break;
    }
    return v;
}

// Enqueue the whole reduction on `st` with working memory at `base` (c.ws.total
// bytes, 256-byte aligned): zero the counters, pack, one stage kernel per
// bandwidth-reduction stage, extract.  Allocates nothing on the device; with
// `timing_allowed` and timing enabled it creates one event pair per stage launch.
// With `vl` the stage kernels also log every reflector there.
static int enqueue_call(const Call& c, const void* band, int64_t ldband, double* d, double* e, hipStream_t st,
                        DeviceState* ds, char* base, bool timing_allowed, const VecLog* vl = nullptr) {
    const Launch& L = c.L;
    const Workspace& ws = c.ws;
    const int64_t n = c.n;
    const int dtype = c.dtype;
    char* W = base;
    int* counters = (int*)(base + ws.band_bytes);
    unsigned* f16_amax = (unsigned*)(counters + ws.off_amax);  // one word per stage
    int* f16_exps = counters + ws.off_exps;                     // nstages + 1 exponents
    int rc = check_hip(bbk::launch_fill(counters, ws.ncounters, 0, st));
    if (!rc) rc = check_hip(bbk::launch_pack(dtype, band, ldband, n, c.b_in, c.bb, W, ws.ldw, ws.uo, 1.0f, st));
    bbp::Stage sg = c.bb > 1 ? bbp::stage_first(c.bb, L.tw) : bbp::Stage{};
    for (int s = 0; s < ws.nstages && !rc; ++s, sg = s < ws.nstages ? bbp::stage_next(sg, L.tw) : sg) {
        bbk::StageArgs a;
        a.W = W;
        a.S = ws.ldw - 1;
        a.uo = ws.uo;
        a.n = (int)n;
        a.b = sg.b;
        a.tw = sg.tw;
        a.c = sg.c;
        a.H = std::max(sg.lag, L.lag);
        a.nsweeps = (int)std::max<int64_t>(n - sg.c - 1, 0);
        a.progress = counters + s * ws.max_sweeps;
        a.claim = counters + ws.off_claim + (kMaxXcd + 1) * s;
        a.abort_flag = a.claim + kMaxXcd;
        a.err_word = ds->err_dev;
        a.spin_limit = spin_limit();
        a.nxcd = ds->nxcd > 1 && L.xcd_run > 0 ? ds->nxcd : 0;
        a.xcd_run = std::max(L.xcd_run, 1);
        a.vlog = vl && vl->base ? vl->base + vl->off[(size_t)s] : nullptr;
        a.wlog = vl ? vl->wlog : 0;
        hipEvent_t done_ev = vl && (size_t)s < vl->stage_done.size() ? vl->stage_done[(size_t)s] : nullptr;
        if (a.nsweeps == 0) {
            if (done_ev) rc = check_hip(hipEventRecord(done_ev, st));
            continue;
        }
        if (dtype == BB_F16) rc = check_hip(bbk::launch_f16_rescale(W, n * ws.ldw, f16_amax + s, f16_exps, s, st));
        if (rc) break;
        const int twm = bbp::kernel_twm(sg.tw);
        int ntl_s = 0, lanes_s = 0;
        stage_shape(L, sg, dtype, &ntl_s, &lanes_s);
        const int64_t ngroups = (a.nsweeps + lanes_s - 1) / lanes_s;
        const int grid = (int)std::min<int64_t>(ngroups, (int64_t)ds->cus * L.groups_per_cu);
        // XCD-aware claims hand group q only to workgroups on XCD (q / xcd_run) mod nxcd,
        // so every XCD must hold a workgroup: the dispatcher deals workgroups to the XCDs
        // round-robin, which a grid of at least nxcd guarantees.  A smaller grid (a band
        // with fewer sweep groups than XCDs) claims in one global order instead.
        if (grid < a.nxcd) a.nxcd = 0;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        bool timed = false;
        if (timing_allowed) {
            std::lock_guard<std::mutex> lk(g_mu);
            timed = g_timing.on;
        }
        if (timed) {
            if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
                if (e0) (void)hipEventDestroy(e0);
                e0 = e1 = nullptr;
                timed = false;
            } else {
                (void)hipEventRecord(e0, st);
            }
        }
        rc = check_hip(bbk::launch_stage(dtype, a, twm, ntl_s, lanes_s, grid, st));
        if (!rc && done_ev) rc = check_hip(hipEventRecord(done_ev, st));
        if (timed) {
            (void)hipEventRecord(e1, st);
            std::lock_guard<std::mutex> lk(g_mu);
            g_timing.events.emplace_back(e0, e1);
        }
    }
    if (!rc) {
        if (dtype == BB_F16) {
            // every stage has n - c - 1 >= 1 sweeps (c <= b - 1 <= n - 2), so each one rescaled
            rc = check_hip(bbk::launch_extract_f16(W, n, ws.ldw, ws.uo, f16_exps, ws.nstages, d, e, st));
        } else {
            rc = check_hip(bbk::launch_extract(dtype, W, n, ws.ldw, ws.uo, 1.0, d, e, st));
        }
    }
    return rc;
}

// Body of bb_reduce for validated arguments, with explicit parameters: working
// memory from the device's stream-ordered pool.
static int reduce_impl(int64_t n, int64_t b, int dtype, const void* band, int64_t ldband, double* d, double* e,
                       hipStream_t st, DeviceState* ds, const bb_params_t& params, bool use_cache) {
    Call c;
    int rc = prepare_call(n, b, dtype, ds, params, use_cache, &c);
    if (rc) return rc;
    void* base = nullptr;
    if (hipMallocAsync(&base, c.ws.total, st) != hipSuccess) return BB_ERR_NOMEM;
    rc = enqueue_call(c, band, ldband, d, e, st, ds, static_cast<char*>(base), true);
    hipError_t fe = hipFreeAsync(base, st);
    if (!rc && fe != hipSuccess) rc = BB_ERR_HIP;
    return rc;
}

// bb_reduce with the device's static scratch as working memory: the same launch
// sequence (counters cleared by a fill kernel, pack, stages, extract), no device
// allocation and no timing events.
int bb_reduce_noalloc(int64_t n, int64_t b, bb_dtype_t dtype, const void* band, int64_t ldband, double* d, double* e,
                      void* stream) {
    if (n < 0) return -1;
    if (b < 0) return -2;
    if (dtype != BB_F64 && dtype != BB_F32 && dtype != BB_F16) return -3;
    if (n > 0 && !band) return -4;
    if (ldband < b + 1) return -5;
    if (n > 0 && !d) return -6;
    if (n > 1 && !e) return -7;
    if (n > (int64_t)1 << 30) return -1;
    if (n == 0) return BB_OK;
    DeviceState* ds = nullptr;
    int rc = device_state(&ds);
    if (rc) return rc;
    Call c;
    rc = prepare_call(n, b, dtype, ds, current_params(), true, &c);
    if (rc) return rc;
    if (c.ws.total > kScratchBytes) return BB_ERR_SCRATCH;
    return enqueue_call(c, band, ldband, d, e, (hipStream_t)stream, ds, ds->scratch_dev, false);
}

// bb_reduce that also forms U and V: the stage kernels log their reflectors in
// stream-ordered working memory, then one back-transformation launch per stage
// applies them to X = I (U from the left reflectors, V from the right ones).
int bb_reduce_vectors(int64_t n, int64_t b, bb_dtype_t dtype, const void* band, int64_t ldband, double* d, double* e,
                      double* U, int64_t ldu, double* V, int64_t ldv, void* stream) {
    if (n < 0 || n > ((int64_t)1 << 30)) return -1;
    if (b < 0) return -2;
    if (dtype != BB_F64 && dtype != BB_F32 && dtype != BB_F16) return -3;
    if (n > 0 && !band) return -4;
    if (ldband < b + 1) return -5;
    if (n > 0 && !d) return -6;
    if (n > 1 && !e) return -7;
    if (U && ldu < std::max<int64_t>(n, 1)) return -9;
    if (V && ldv < std::max<int64_t>(n, 1)) return -11;
    if (n == 0) return BB_OK;
    DeviceState* ds = nullptr;
    int rc = device_state(&ds);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    Call c;
    rc = prepare_call(n, b, dtype, ds, current_params(), true, &c);
    if (rc) return rc;
    VecLog vl = veclog_layout(n, c.bb, c.L.tw);
    // The back-transformation of stage s needs only stage s's reflector log (and the
    // factors after stage s-1's), so it runs on a second stream while the reduction
    // goes on with stage s+1: the stage kernels are latency-bound and leave most of
    // the chip to it.  Events order the two streams (fork after the work already on
    // `stream`, one event per stage, join before the workspace is freed), which also
    // holds under stream capture.
    hipStream_t aux = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        if (!ds->aux && hipStreamCreateWithFlags(&ds->aux, hipStreamNonBlocking) != hipSuccess) ds->aux = nullptr;
        aux = ds->aux;
    }
    if (!aux) return BB_ERR_HIP;
    const size_t nst = vl.off.size();
    std::vector<hipEvent_t> evs(nst + 2, nullptr);  // stage events, fork, join
    auto destroy_events = [&]() {
        for (hipEvent_t ev : evs)
            if (ev) (void)hipEventDestroy(ev);
    };
    for (hipEvent_t& ev : evs)
        if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
            ev = nullptr;
            destroy_events();
            return BB_ERR_HIP;
        }
    const size_t total = c.ws.total + align_up(sizeof(double) * (size_t)vl.doubles, 256);
    void* base = nullptr;
    if (hipMallocAsync(&base, total, st) != hipSuccess) {
        destroy_events();
        return BB_ERR_NOMEM;
    }
    vl.base = vl.doubles > 0 ? reinterpret_cast<double*>(static_cast<char*>(base) + c.ws.total) : nullptr;
    vl.stage_done.assign(evs.begin(), evs.begin() + nst);
    hipEvent_t fork = evs[nst], join = evs[nst + 1];
    rc = check_hip(hipEventRecord(fork, st));
    const bool forked = !rc && hipStreamWaitEvent(aux, fork, 0) == hipSuccess;
    if (!forked && !rc) rc = BB_ERR_HIP;
    if (!rc && U) rc = check_hip(bbk::launch_identity(U, n, ldu, aux));
    if (!rc && V) rc = check_hip(bbk::launch_identity(V, n, ldv, aux));
    if (!rc) rc = enqueue_call(c, band, ldband, d, e, st, ds, static_cast<char*>(base), true, &vl);
    if (!rc && vl.base) {
        size_t s = 0;
        for (bbp::Stage sg = bbp::stage_first(c.bb, c.L.tw); !rc && s < nst; sg = bbp::stage_next(sg, c.L.tw), ++s) {
            const int nsw = (int)std::max<int64_t>(n - sg.c - 1, 0);
            rc = check_hip(hipStreamWaitEvent(aux, vl.stage_done[s], 0));
            if (!rc)
                rc = check_hip(bbk::launch_backtransform(V, ldv, U, ldu, (int)n, sg.b, sg.tw, sg.c, nsw,
                                                         vl.nsteps[s], vl.base + vl.off[s], vl.wlog, aux));
            if (sg.c <= 1) break;
        }
    }
    if (forked) {  // always joined, so that nothing on `aux` outlives the workspace
        const int jr = check_hip(hipEventRecord(join, aux));
        const int jw = jr ? jr : check_hip(hipStreamWaitEvent(st, join, 0));
        if (!rc) rc = jw;
    }
    hipError_t fe = hipFreeAsync(base, st);
    if (!rc && fe != hipSuccess) rc = BB_ERR_HIP;
    destroy_events();
    return rc;
}

int bb_sym_min_lag(int64_t c) { return c < 1 ? -1 : (c == 1 ? 3 : 2); }

double bb_sym_model_bytes(int64_t n, int64_t b, int elem_size, int tw) {
    if (n <= 0 || b < 0 || elem_size <= 0 || tw < 1) return 0.0;
    return bbp::sym_model_bytes(n, std::min<int64_t>(b, n - 1), elem_size, tw);
}

// Symmetric band -> tridiagonal: pack the lower band into a working band with
// room for the bulge fill, one persistent stage kernel per bandwidth-reduction
// stage, extract the diagonal and sub-diagonal.
int bb_sym_reduce(int64_t n, int64_t b, bb_dtype_t dtype, const void* band, int64_t ldband, double* d, double* e,
                  void* stream) {
    if (n < 0 || n > ((int64_t)1 << 30)) return -1;
    if (b < 0) return -2;
    if (dtype != BB_F64 && dtype != BB_F32 && dtype != BB_F16) return -3;
    if (n > 0 && !band) return -4;
    if (ldband < b + 1) return -5;
    if (n > 0 && !d) return -6;
    if (n > 1 && !e) return -7;
    if (n == 0) return BB_OK;
    if (dtype == BB_F16) return BB_ERR_UNSUPPORTED;
    DeviceState* ds = nullptr;
    int rc = device_state(&ds);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    const bb_params_t prm = current_params();
    const int64_t bb = std::min<int64_t>(b, n - 1);
    const int tw = prm.tw ? prm.tw : bbp::default_tw(dtype);
    if (tw < 1 || tw > 32) return BB_ERR_UNSUPPORTED;
    const int tw0 = bb > 1 ? bbp::stage_first(bb, tw).tw : 0;
    const int64_t ldw = (int64_t)align_up((size_t)(bb + tw0 + 2), 2);
    const int nstages = bbp::stage_count(bb, tw);
    const size_t band_bytes = align_up((size_t)n * (size_t)ldw * elem_size(dtype), 256);
    const int64_t per_stage = n + 2;  // progress words, claim, abort
    const size_t total = band_bytes + align_up(sizeof(int) * (size_t)(per_stage * std::max(nstages, 1)), 256);
    void* base = nullptr;
    if (hipMallocAsync(&base, total, st) != hipSuccess) return BB_ERR_NOMEM;
    char* W = static_cast<char*>(base);
    int* counters = reinterpret_cast<int*>(W + band_bytes);
    rc = check_hip(bbk::launch_fill(counters, per_stage * std::max(nstages, 1), 0, st));
    if (!rc) rc = check_hip(bbk::launch_sym_pack(dtype, band, ldband, n, bb, W, ldw, st));
    // workgroups per CU: as many as fit (a 512-thread workgroup of the FP64 32-wide step
    // uses 234 registers per lane, so one; two of 256 threads)
    if (bb > 1) {
        int s = 0;
        for (bbp::Stage sg = bbp::stage_first(bb, tw); !rc; sg = bbp::stage_next(sg, tw), ++s) {
            bbk::SymStageArgs a;
            a.W = W;
            a.ldw = ldw;
            a.n = (int)n;
            a.b = sg.b;
            a.tw = sg.tw;
            a.c = sg.c;
            a.H = std::max(bb_sym_min_lag(sg.c), prm.lag);
            a.nsweeps = (int)std::max<int64_t>(n - sg.c - 1, 0);
            a.progress = counters + per_stage * s;
            a.claim = a.progress + n;
            a.abort_flag = a.claim + 1;
            a.err_word = ds->err_dev;
            a.spin_limit = spin_limit();
            if (a.nsweeps > 0) {
                const int nt = bbk::sym_stage_threads(sg.b, sg.tw);
                const int gpc = prm.groups_per_cu ? prm.groups_per_cu : (nt == 256 ? 2 : 1);
                const int grid = (int)std::min<int64_t>(a.nsweeps, (int64_t)ds->cus * gpc);
                rc = check_hip(bbk::launch_sym_stage(dtype, a, bbp::kernel_twm(sg.tw), nt, grid, st));
            }
            if (sg.c <= 1) break;
        }
    }
    if (!rc) rc = check_hip(bbk::launch_sym_extract(dtype, W, n, ldw, d, e, st));
    hipError_t fe = hipFreeAsync(base, st);
    if (!rc && fe != hipSuccess) rc = BB_ERR_HIP;
    return rc;
}

int bb_reduce_batched(int64_t count, const int64_t* n, const int64_t* b, bb_dtype_t dtype, const void* const* band,
                      const int64_t* ldband, double* const* d, double* const* e, void* stream) {
    if (count < 0 || count > (1 << 20)) return -1;
    if (count > 0 && (!n || !b || !band || !ldband || !d || !e))
        return !n ? -2 : !b ? -3 : !band ? -5 : !ldband ? -6 : !d ? -7 : -8;
    if (dtype != BB_F64 && dtype != BB_F32 && dtype != BB_F16) return -4;
    for (int64_t i = 0; i < count; ++i) {
        if (n[i] < 0 || n[i] > (int64_t)1 << 30) return -2;
        if (b[i] < 0) return -3;
        if (n[i] > 0 && !band[i]) return -5;
        if (ldband[i] < b[i] + 1) return -6;
        if (n[i] > 0 && !d[i]) return -7;
        if (n[i] > 1 && !e[i]) return -8;
    }
    if (count == 0) return BB_OK;
    hipStream_t st = (hipStream_t)stream;
    DeviceState* ds = nullptr;
    int rc = device_state(&ds);
    if (rc) return rc;
    int64_t max_n = 0, max_b = 0;
    for (int64_t i = 0; i < count; ++i) {
        max_n = std::max(max_n, n[i]);
        max_b = std::max(max_b, std::min(b[i], std::max<int64_t>(n[i] - 1, 0)));
    }
    // a nonzero bb_set_params field wins, then a bb_autotune_batched entry for this
    // exact batch, then the batched defaults
    bb_params_t prm = current_params();
    bb_params_t tuned;
    if (batch_tuned_lookup(count, n, b, dtype, &tuned)) {
        if (!prm.tw) prm.tw = tuned.tw;
        if (!prm.threads_per_window) prm.threads_per_window = tuned.threads_per_window;
        if (!prm.sweeps_per_group) prm.sweeps_per_group = tuned.sweeps_per_group;
        if (!prm.groups_per_cu) prm.groups_per_cu = tuned.groups_per_cu;
        if (!prm.lag) prm.lag = tuned.lag;
        if (!prm.xcd_run) prm.xcd_run = tuned.xcd_run;
    }
    Launch L = resolve(max_n, max_b, dtype, ds->lds_per_block, prm, false, 4);
    if (L.tw < 1 || L.tw > bbp::max_tw(dtype)) return BB_ERR_UNSUPPORTED;
    BatchPlan* bp = nullptr;
    rc = batch_plan(count, n, b, dtype, L, st, &bp);
    if (rc) return rc;
    return batch_run(bp, ds, band, ldband, d, e, L, st);
}

int bb_set_params(const bb_params_t* p) {
    bb_params_t q = {0, 0, 0, 0, 0, 0};
    if (p) {
        if (p->tw < 0 || p->tw > bbp::kMaxTW) return -1;
        if (p->threads_per_window != 0 && p->threads_per_window != 64 && p->threads_per_window != 128 &&
            p->threads_per_window != 256)
            return -1;
        if (p->sweeps_per_group < 0 || p->sweeps_per_group > 16) return -1;
        if (p->threads_per_window && p->sweeps_per_group && p->threads_per_window * p->sweeps_per_group > 1024)
            return -1;
        if (p->groups_per_cu < 0 || p->groups_per_cu > 16) return -1;
        if (p->lag < 0 || p->lag > 64) return -1;
        if (p->xcd_run < 0 || p->xcd_run > 4096) return -1;
        q = *p;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    g_params = q;
    return BB_OK;
}

int bb_get_params(bb_params_t* p) {
    if (!p) return -1;
    std::lock_guard<std::mutex> lk(g_mu);
    *p = g_params;
    return BB_OK;
}

size_t bb_workspace_bytes(int64_t n, int64_t b, bb_dtype_t dtype) {
    if (n <= 0 || b < 0) return 0;
    const int64_t bb = std::min<int64_t>(b, n - 1);
    Launch L = resolve(n, bb, dtype, 65536, current_params());
    return workspace_layout(n, bb, dtype, L.tw).total;
}

double bb_model_bytes(int64_t n, int64_t b, int elem_size, int tw) {
    if (n <= 0 || b < 0 || elem_size <= 0 || tw < 1) return 0.0;
    return bbp::model_bytes(n, std::min<int64_t>(b, n - 1), elem_size, tw);
}

int bb_plan(int64_t b, int tw, int max_stages, int* bs, int* tws, int* cs, int* lags) {
    if (b < 0) return -1;
    if (tw < 1) return -2;
    if (max_stages < 0) return -3;
    bbp::Plan plan = bbp::make_plan(b, tw);
    for (int s = 0; s < (int)plan.stages.size() && s < max_stages; ++s) {
        if (bs) bs[s] = plan.stages[s].b;
        if (tws) tws[s] = plan.stages[s].tw;
        if (cs) cs[s] = plan.stages[s].c;
        if (lags) lags[s] = plan.stages[s].lag;
    }
    return (int)plan.stages.size();
}

int bb_min_lag(int64_t c) { return c < 1 ? -1 : bbp::min_lag((int)std::min<int64_t>(c, 1 << 20)); }

int bb_bidiag_sigma(int64_t n, const double* d, const double* e, double* sigma, void* stream) {
    if (n < 0 || n > (int64_t(1) << 29)) return -1;
    if (n > 0 && !d) return -2;
    if (n > 1 && !e) return -3;
    if (n > 0 && !sigma) return -4;
    if (n == 0) return BB_OK;
    DeviceState* ds = nullptr;
    int rc = device_state(&ds);
    if (rc) return rc;
    return check_hip(bbk::launch_bidiag_sigma(d, e, n, sigma, (hipStream_t)stream));
}

int bb_stream_status(void* stream) {
    DeviceState* ds = nullptr;
    int rc = device_state(&ds);
    if (rc) return rc;
    if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return BB_ERR_HIP;
    return read_err_word(ds, true);
}

int bb_timing_enable(int on) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_timing.on = on != 0;
    return BB_OK;
}

int bb_timing_read(double* stage_ms, int64_t* stage_launches) {
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        ev.swap(g_timing.events);
    }
    double tot = 0.0;
    int rc = BB_OK;
    for (auto& pr : ev) {
        float ms = 0.f;
        if (hipEventSynchronize(pr.second) != hipSuccess || hipEventElapsedTime(&ms, pr.first, pr.second) != hipSuccess)
            rc = BB_ERR_HIP;
        tot += ms;
        hipEventDestroy(pr.first);
        hipEventDestroy(pr.second);
    }
    if (stage_ms) *stage_ms = tot;
    if (stage_launches) *stage_launches = (int64_t)ev.size();
    return rc;
}

int bb_release(void) {
    bbp::autotune_clear();
    {
        std::lock_guard<std::mutex> lk(g_mu);
        g_batch_tuned.clear();
    }
    batch_plans_clear();
    return BB_OK;
}

const char* bb_error_string(int code) {
    if (code < 0) return "invalid argument";
    switch (code) {
        case BB_OK: return "success";
        case BB_ERR_HIP: return "HIP runtime error";
        case BB_ERR_TIMEOUT: return "device watchdog: dependency wait timed out";
        case BB_ERR_NOMEM: return "out of memory";
        case BB_ERR_UNSUPPORTED: return "unsupported parameters";
        case BB_ERR_NODEVICE: return "no usable device";
        case BB_ERR_SCRATCH: return "working memory exceeds the 64 MiB static scratch of bb_reduce_noalloc";
        default: return "unknown error";
    }
}

}  // extern "C"

// Critical-path model used to rank autotune candidates: per stage, lag * (n - c)
// half-steps, each costing a fixed latency plus a term growing with the window.
static double model_time(int64_t n, int64_t b, int elem, int tw) {
    double t = 0.0;
    for (const bbp::Stage& s : bbp::make_plan(b, tw).stages)
        t += (double)s.lag * (double)(n - s.c) * (1.0 + (double)elem * (s.b + s.tw) * (s.tw + 1) / 16384.0);
    return t;
}

namespace {

constexpr int kTuneReps = 3;          // timed runs per candidate (the median decides)
constexpr float kTuneMargin = 0.99f;  // a candidate replaces the defaults only if at least 1 % faster

// Candidate launch parameters: the built-in defaults first, then shapes that win
// in some regime.  Fields fixed by bb_set_params hold for every candidate.
std::vector<bb_params_t> tune_candidates(int dtype, bool batched, const bb_params_t& user) {
    const int tw_alt = dtype == BB_F64 ? 16 : 64;
    std::vector<bb_params_t> c;
    if (!batched)
        c = {{0, 0, 0, 0, 0, 0},      {tw_alt, 0, 0, 0, 0, 0}, {0, 0, 0, 1, 0, 0}, {0, 0, 0, 3, 0, 0},
             {0, 0, 0, 0, 0, 1},      {0, 0, 0, 0, 0, 8},      {0, 0, 2, 0, 0, 0}, {0, 128, 1, 2, 0, 0}};
    else
        c = {{0, 0, 0, 0, 0, 0}, {tw_alt, 0, 0, 0, 0, 0}, {0, 0, 0, 2, 0, 0}, {0, 0, 0, 3, 0, 0},
             {tw_alt, 0, 0, 3, 0, 0}, {0, 128, 0, 0, 0, 0}, {0, 0, 2, 2, 0, 0}};
    std::vector<bb_params_t> out;
    for (bb_params_t x : c) {
        if (user.tw) x.tw = user.tw;
        if (user.threads_per_window) x.threads_per_window = user.threads_per_window;
        if (user.sweeps_per_group) x.sweeps_per_group = user.sweeps_per_group;
        if (user.groups_per_cu) x.groups_per_cu = user.groups_per_cu;
        if (user.lag) x.lag = user.lag;
        if (user.xcd_run) x.xcd_run = user.xcd_run;
        if (x.tw > bbp::max_tw(dtype)) continue;
        bool dup = false;
        for (const bb_params_t& y : out)
            if (!std::memcmp(&x, &y, sizeof(x))) dup = true;
        if (!dup) out.push_back(x);
    }
    return out;
}

// Time `run` (which enqueues one call on st) kReps times after one untimed run;
// *ms receives the median.
template <typename Run>
int time_median(Run&& run, hipStream_t st, DeviceState* ds, hipEvent_t e0, hipEvent_t e1, float* ms) {
    int rc = run();
    if (!rc) rc = check_hip(hipStreamSynchronize(st));
    float t[kTuneReps];
    for (int i = 0; i < kTuneReps && !rc; ++i) {
        rc = check_hip(hipEventRecord(e0, st));
        if (!rc) rc = run();
        if (!rc) rc = check_hip(hipEventRecord(e1, st));
        if (!rc) rc = check_hip(hipEventSynchronize(e1));
        if (!rc) rc = check_hip(hipEventElapsedTime(&t[i], e0, e1));
    }
    if (!rc && read_err_word(ds, false)) rc = BB_ERR_TIMEOUT;
    if (rc) return rc;
    std::sort(t, t + kTuneReps);
    *ms = t[kTuneReps / 2];
    return BB_OK;
}

// Pick among timed candidates: the fastest median, unless it is not at least
// 1 % faster than the defaults (candidate 0), which then stay.
size_t pick_winner(const std::vector<float>& ms) {
    size_t best = 0;
    for (size_t i = 1; i < ms.size(); ++i)
        if (ms[i] < ms[best]) best = i;
    return ms[best] <= kTuneMargin * ms[0] ? best : 0;
}

// Free batch plans made after index `from` whose launch does not match `keep`.
void batch_plans_drop_after(size_t from, const BatchPlan* keep) {
    std::lock_guard<std::mutex> lk(g_mu);
    std::vector<BatchPlan*> kept(g_batch_plans.begin(), g_batch_plans.begin() + std::min(from, g_batch_plans.size()));
    for (size_t i = from; i < g_batch_plans.size(); ++i) {
        BatchPlan* p = g_batch_plans[i];
        if (p == keep) {
            kept.push_back(p);
            continue;
        }
        if (p->staged_pending) (void)hipEventSynchronize(p->staged);
        (void)hipEventDestroy(p->staged);
        (void)hipHostFree(p->pinned);
        (void)hipHostFree(p->pinned_capture);
        (void)hipFree(p->dev);
        delete p;
    }
    g_batch_plans.swap(kept);
}

}  // namespace

extern "C" int bb_autotune(int64_t n, int64_t b, bb_dtype_t dtype, void* stream, bb_params_t* out) {
    if (n < 0) return -1;
    if (b < 0) return -2;
    if (dtype != BB_F64 && dtype != BB_F32 && dtype != BB_F16) return -3;
    DeviceState* ds = nullptr;
    int rc = device_state(&ds);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    const int64_t bb = std::min<int64_t>(b, std::max<int64_t>(n - 1, 0));
    const bb_params_t user = current_params();
    auto report = [&](const bb_params_t& p) {
        Launch L = resolve(n, bb, dtype, ds->lds_per_block, p, false);
        if (out) *out = bb_params_t{L.tw, L.ntl, L.lanes, L.groups_per_cu, L.lag, L.xcd_run};
    };
    if (n < 64 || bb <= 1) {  // nothing worth timing
        report(user);
        return BB_OK;
    }
    const int64_t nt = std::min<int64_t>(n, 32768);
    const int64_t bt = std::min<int64_t>(bb, nt - 1);
    const int elem = (int)elem_size(dtype);
    // rank by the critical-path model; the defaults (first) are always timed
    std::vector<bb_params_t> cands = tune_candidates(dtype, false, user);
    auto model = [&](const bb_params_t& c) {
        const int tw = c.tw ? c.tw : bbp::default_tw(dtype);
        return model_time(nt, bt, elem, (int)std::min<int64_t>(tw, std::max<int64_t>(bt - 1, 1)));
    };
    std::stable_sort(cands.begin() + 1, cands.end(),
                     [&](const bb_params_t& x, const bb_params_t& y) { return model(x) < model(y) * 0.999; });
    if (cands.size() > 6) cands.resize(6);
    // synthetic band of the (capped) shape, timed on `stream`
    void *band = nullptr, *dbuf = nullptr;
    const size_t band_bytes = (size_t)nt * (size_t)(bt + 1) * (size_t)elem;
    if (hipMallocAsync(&band, band_bytes, st) != hipSuccess) return BB_ERR_NOMEM;
    if (hipMallocAsync(&dbuf, sizeof(double) * 2 * (size_t)nt, st) != hipSuccess) {
        (void)hipFreeAsync(band, st);
        return BB_ERR_NOMEM;
    }
    double* d = static_cast<double*>(dbuf);
    double* e = d + nt;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    rc = check_hip(bbk::launch_fill_synth(dtype, band, (int64_t)(band_bytes / elem), 0x5eed, st));
    if (!rc) rc = check_hip(hipEventCreate(&e0));
    if (!rc) rc = check_hip(hipEventCreate(&e1));
    std::vector<float> ms;
    for (size_t i = 0; i < cands.size() && !rc; ++i) {
        float t = 0.f;
        rc = time_median([&] { return reduce_impl(nt, bt, dtype, band, bt + 1, d, e, st, ds, cands[i], false); }, st,
                         ds, e0, e1, &t);
        ms.push_back(t);
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFreeAsync(dbuf, st);
    (void)hipFreeAsync(band, st);
    if (hipStreamSynchronize(st) != hipSuccess && !rc) rc = BB_ERR_HIP;
    if (rc) return rc;
    const bb_params_t best = cands[pick_winner(ms)];
    bbp::autotune_store(n, bb, dtype, bbp::Tuned{best});
    report(best);
    return BB_OK;
}

extern "C" int bb_autotune_batched(int64_t count, const int64_t* n, const int64_t* b, bb_dtype_t dtype, void* stream,
                                   bb_params_t* out) {
    if (count < 0 || count > (1 << 20)) return -1;
    if (count > 0 && (!n || !b)) return !n ? -2 : -3;
    if (dtype != BB_F64 && dtype != BB_F32 && dtype != BB_F16) return -4;
    for (int64_t i = 0; i < count; ++i) {
        if (n[i] < 0 || n[i] > (int64_t)1 << 30) return -2;
        if (b[i] < 0) return -3;
    }
    DeviceState* ds = nullptr;
    int rc = device_state(&ds);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    const bb_params_t user = current_params();
    int64_t max_n = 0, max_b = 0;
    for (int64_t i = 0; i < count; ++i) {
        max_n = std::max(max_n, n[i]);
        max_b = std::max(max_b, std::min(b[i], std::max<int64_t>(n[i] - 1, 0)));
    }
    auto report = [&](const bb_params_t& p) {
        Launch L = resolve(max_n, max_b, dtype, ds->lds_per_block, p, false, 4);
        if (out) *out = bb_params_t{L.tw, L.ntl, L.lanes, L.groups_per_cu, L.lag, L.xcd_run};
    };
    if (count == 0 || max_n < 2) {
        report(user);
        return BB_OK;
    }
    // synthetic bands of the batch's shapes (one buffer), outputs, pointer arrays
    const size_t elem = elem_size(dtype);
    std::vector<size_t> off((size_t)count);
    size_t tot = 0, tot_d = 0;
    for (int64_t i = 0; i < count; ++i) {
        off[(size_t)i] = tot;
        tot += align_up((size_t)std::max<int64_t>(n[i], 1) * (size_t)(b[i] + 1) * elem, 256);
        tot_d += 2 * (size_t)std::max<int64_t>(n[i], 1);
    }
    void *bands = nullptr, *dbuf = nullptr;
    if (hipMallocAsync(&bands, tot, st) != hipSuccess) return BB_ERR_NOMEM;
    if (hipMallocAsync(&dbuf, sizeof(double) * tot_d, st) != hipSuccess) {
        (void)hipFreeAsync(bands, st);
        return BB_ERR_NOMEM;
    }
    std::vector<const void*> bp((size_t)count);
    std::vector<int64_t> ld((size_t)count);
    std::vector<double*> dp((size_t)count), ep((size_t)count);
    double* dd = static_cast<double*>(dbuf);
    for (int64_t i = 0; i < count; ++i) {
        bp[(size_t)i] = static_cast<char*>(bands) + off[(size_t)i];
        ld[(size_t)i] = b[i] + 1;
        dp[(size_t)i] = dd;
        ep[(size_t)i] = dd + std::max<int64_t>(n[i], 1);
        dd += 2 * (size_t)std::max<int64_t>(n[i], 1);
    }
    rc = check_hip(bbk::launch_fill_synth((int)dtype, bands, (int64_t)(tot / elem), 0xba7c, st));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (!rc) rc = check_hip(hipEventCreate(&e0));
    if (!rc) rc = check_hip(hipEventCreate(&e1));
    size_t nplans0 = 0;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        nplans0 = g_batch_plans.size();
    }
    const std::vector<bb_params_t> cands = tune_candidates(dtype, true, user);
    std::vector<float> ms;
    std::vector<BatchPlan*> plans;
    for (size_t i = 0; i < cands.size() && !rc; ++i) {
        Launch L = resolve(max_n, max_b, dtype, ds->lds_per_block, cands[i], false, 4);
        BatchPlan* P = nullptr;
        if (L.tw < 1 || L.tw > bbp::max_tw(dtype)) rc = BB_ERR_UNSUPPORTED;
        if (!rc) rc = batch_plan(count, n, b, dtype, L, st, &P);
        float t = 0.f;
        if (!rc)
            rc = time_median([&] { return batch_run(P, ds, bp.data(), ld.data(), dp.data(), ep.data(), L, st); }, st,
                             ds, e0, e1, &t);
        ms.push_back(t);
        plans.push_back(P);
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFreeAsync(dbuf, st);
    (void)hipFreeAsync(bands, st);
    if (hipStreamSynchronize(st) != hipSuccess && !rc) rc = BB_ERR_HIP;
    if (rc) {
        batch_plans_drop_after(nplans0, nullptr);
        return rc;
    }
    const size_t w = pick_winner(ms);
    batch_plans_drop_after(nplans0, plans[w]);  // the winner's plan serves the caller's next calls
    batch_tuned_store(count, n, b, dtype, cands[w]);
    report(cands[w]);
    return BB_OK;
}

extern "C" int bb_resolved_params(int64_t n, int64_t b, bb_dtype_t dtype, bb_params_t* out) {
    if (n < 0) return -1;
    if (b < 0) return -2;
    if (dtype != BB_F64 && dtype != BB_F32 && dtype != BB_F16) return -3;
    if (!out) return -4;
    DeviceState* ds = nullptr;
    const size_t lds = device_state(&ds) == BB_OK ? ds->lds_per_block : 65536;
    Launch L = resolve(n, std::min<int64_t>(b, std::max<int64_t>(n - 1, 0)), dtype, lds, current_params());
    *out = bb_params_t{L.tw, L.ntl, L.lanes, L.groups_per_cu, L.lag, L.xcd_run};
    return BB_OK;
}
