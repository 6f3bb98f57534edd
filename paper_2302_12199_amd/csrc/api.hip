// C ABI of the MSF library: argument checks, workspace handling, the
// kernel-timing profiler and dispatch to the Borůvka / Filter-Borůvka drivers.
// Every step of the computation runs in the HIP kernels; the host only sizes
// launches from small counter blocks read back between them.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <mutex>
#include <vector>

#include "engine.h"
#include "filter.h"

namespace msf {

// ------------------------------------------------------------- error text
namespace {
thread_local char g_err[512];
}
void set_err(const char* what, hipError_t e) {
    snprintf(g_err, sizeof g_err, "%s: %s", what, hipGetErrorString(e));
}
void set_err_text(const char* text) { snprintf(g_err, sizeof g_err, "%s", text); }
const char* last_err() { return g_err; }

// ------------------------------------------------------------ kernel timing
namespace {
const char* const kKernelNames[K_COUNT] = {
    "minedge_r0", "hook", "jump", "scan_roots", "label", "pass", "compact", "compose",
    "fill", "scan_prep", "sample", "partition", "filter", "rep_maint", "mlp", "batch", "tail",
    "pass_r0", "bucket_index", "bucket_scatter", "bucket_min", "bucket_label", "bucket_pass",
    "dedup"};

struct Profiler {
    std::mutex mu;
    bool on = false;
    uint64_t launches[K_COUNT] = {};
    double ms[K_COUNT] = {};
    double bytes[K_COUNT] = {};
    struct Pending { int kid; hipEvent_t a, b; double bytes; };
    std::vector<Pending> pending;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pool;
};
Profiler g_prof;
}  // namespace

bool prof_on() {
    std::lock_guard<std::mutex> l(g_prof.mu);
    return g_prof.on;
}

namespace {
thread_local bool t_prof_off = false;   // set for calls that must create no events
}

int prof_begin(int kid, hipStream_t s) {
    if (t_prof_off) return -1;
    std::lock_guard<std::mutex> l(g_prof.mu);
    if (!g_prof.on) return -1;
    std::pair<hipEvent_t, hipEvent_t> ev;
    if (!g_prof.pool.empty()) {
        ev = g_prof.pool.back();
        g_prof.pool.pop_back();
    } else if (hipEventCreate(&ev.first) != hipSuccess ||
               hipEventCreate(&ev.second) != hipSuccess) {
        return -1;
    }
    (void)hipEventRecord(ev.first, s);
    g_prof.pending.push_back({kid, ev.first, ev.second, 0.0});
    return (int)g_prof.pending.size() - 1;
}

void prof_end(int h, hipStream_t s, double bytes) {
    if (h < 0) return;
    std::lock_guard<std::mutex> l(g_prof.mu);
    if (h >= (int)g_prof.pending.size()) return;
    (void)hipEventRecord(g_prof.pending[h].b, s);
    g_prof.pending[h].bytes += bytes;
}

void prof_add(int kid, double bytes) {
    std::lock_guard<std::mutex> l(g_prof.mu);
    if (g_prof.on) g_prof.bytes[kid] += bytes;
}

// Resolves the launches whose end event has completed; launches of calls
// still running on other streams stay pending.
void prof_resolve() {
    std::lock_guard<std::mutex> l(g_prof.mu);
    size_t keep = 0;
    for (size_t i = 0; i < g_prof.pending.size(); ++i) {
        auto& p = g_prof.pending[i];
        if (hipEventQuery(p.b) == hipErrorNotReady) {
            g_prof.pending[keep++] = p;
            continue;
        }
        float t = 0.f;
        if (hipEventElapsedTime(&t, p.a, p.b) == hipSuccess) {
            g_prof.launches[p.kid] += 1;
            g_prof.ms[p.kid] += t;
            g_prof.bytes[p.kid] += p.bytes;
        }
        (void)hipGetLastError();
        g_prof.pool.push_back({p.a, p.b});
    }
    g_prof.pending.resize(keep);
}

// ------------------------------------------------------- counter read-back
// Every call reads the device control block into a host block of its own, so
// calls on different streams (or threads) run side by side: msf_compute takes
// a pinned block from a pool (allocated on first need, kept for reuse),
// msf_compute_noalloc reads into ordinary host memory.
namespace {
std::mutex g_pool_mu;
std::vector<Ctrl*> g_pinned_free;
thread_local Ctrl* t_host_ctrl = nullptr;

int take_pinned_ctrl(Ctrl** out) {
    {
        std::lock_guard<std::mutex> l(g_pool_mu);
        if (!g_pinned_free.empty()) {
            *out = g_pinned_free.back();
            g_pinned_free.pop_back();
            return MSF_OK;
        }
    }
    HIP_TRY(hipHostMalloc((void**)out, sizeof(Ctrl), hipHostMallocDefault));
    return MSF_OK;
}

void give_pinned_ctrl(Ctrl* c) {
    std::lock_guard<std::mutex> l(g_pool_mu);
    g_pinned_free.push_back(c);
}
}  // namespace

Ctrl* host_ctrl() { return t_host_ctrl; }

int read_ctrl(const Ctrl* dctrl, Ctrl* host, hipStream_t s) {
    HIP_TRY(hipMemcpyAsync(host, dctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    prof_resolve();
    return MSF_OK;
}

}  // namespace msf

using namespace msf;

namespace {

int check_args(const int32_t* u, const int32_t* v, const uint32_t* w, int64_t m, int64_t n,
               const uint8_t* mask, const uint64_t* total, const msf_options* opt) {
    if (n < 0 || n > 0x7fffffffLL || m < 0 || m > 0xffffffffLL) return MSF_EINVAL;
    if (n == 0 && m != 0) return MSF_EINVAL;
    if (!total) return MSF_EINVAL;
    if (m > 0 && (!u || !v || !w || !mask)) return MSF_EINVAL;
    if (opt) {
        if (opt->algo != MSF_ALGO_BORUVKA && opt->algo != MSF_ALGO_FILTER) return MSF_EINVAL;
        if (opt->pivot < MSF_PIVOT_MEDIAN || opt->pivot > MSF_PIVOT_MLP) return MSF_EINVAL;
        if (!(opt->quantile >= 0.0f && opt->quantile <= 1.0f)) return MSF_EINVAL;
        if (opt->sample_size < 0 || opt->sample_size > 8192) return MSF_EINVAL;
        if (opt->sparse_degree < 0 || opt->min_split_edges < 0) return MSF_EINVAL;
        if (opt->round0 < MSF_ROUND0_AUTO || opt->round0 > MSF_ROUND0_BUCKETS) return MSF_EINVAL;
        if (opt->dedup_policy < MSF_DEDUP_AUTO || opt->dedup_policy > MSF_DEDUP_LOCAL)
            return MSF_EINVAL;
        if (opt->split_retries < 0 || opt->split_retries > 64 || opt->defer_edges < 0)
            return MSF_EINVAL;
        if (opt->tail_threshold < 0 || opt->tail_threshold > kTailMax) return MSF_EINVAL;
        for (int i = 0; i < 3; ++i)
            if (opt->reserved[i]) return MSF_EINVAL;
    }
    return MSF_OK;
}

bool use_filter(const msf_options* opt) { return opt && opt->algo == MSF_ALGO_FILTER; }
bool round0_buckets(const msf_options* opt) { return !opt || opt->round0 != MSF_ROUND0_EDGES; }
bool exact_dedup(const msf_options* opt) { return opt && opt->dedup_policy == MSF_DEDUP_EXACT; }

// `hc`: the host block this call reads the device counters into.
int solve(const int32_t* u, const int32_t* v, const uint32_t* w, int64_t m, int64_t n,
          uint8_t* mask, uint64_t* total_out, char* ws, hipStream_t s, const msf_options* opt,
          msf_stats* stats, Ctrl* hc) {
    struct Bind {
        explicit Bind(Ctrl* c) { t_host_ctrl = c; }
        ~Bind() { t_host_ctrl = nullptr; }
    } bind(hc);
    msf_stats local;
    memset(&local, 0, sizeof local);
    msf_stats* st = stats ? stats : &local;
    int rc;
    if (use_filter(opt)) {
        rc = filter_solve(u, v, w, m, n, mask, ws, s, *opt, st);
    } else {
        EngineBuffers B;
        engine_carve(ws, m, n, &B, round0_buckets(opt), exact_dedup(opt));
        B.round0 = opt ? opt->round0 : MSF_ROUND0_AUTO;
        B.dedup = opt ? opt->dedup_policy : MSF_DEDUP_AUTO;
        B.tail = opt ? opt->tail_threshold : 0;
        launch_zero_bytes((uint8_t*)B.ctrl, sizeof(Ctrl), s);
        int h = prof_begin(K_FILL, s);
        launch_zero_bytes(mask, m, s);
        prof_end(h, s, (double)m);
        View g{u, v, nullptr, w, nullptr, m};
        rc = engine_solve(B, kOrig, g, n, mask, nullptr, s, st);
        if (rc == MSF_OK) {
            rc = read_ctrl(B.ctrl, hc, s);
            st->total_weight = hc->total;
            st->msf_edges = hc->msf_edges;
            st->base_cases = 1;
        }
    }
    if (rc == MSF_OK) *total_out = st->total_weight;
    return rc;
}

}  // namespace

extern "C" {

size_t msf_workspace_bytes(int64_t m, int64_t n, const msf_options* opt) {
    if (m < 0 || n < 0) return 0;
    return use_filter(opt) ? filter_bytes(m, n, *opt)
                           : engine_bytes(m, n, round0_buckets(opt), exact_dedup(opt));
}

int msf_compute(const int32_t* u, const int32_t* v, const uint32_t* w, int64_t m, int64_t n,
                uint8_t* mask_out, uint64_t* total_weight_out, void* workspace,
                size_t workspace_bytes, void* stream, const msf_options* opt,
                msf_stats* stats) {
    int st = check_args(u, v, w, m, n, mask_out, total_weight_out, opt);
    if (st) return st;
    if (stats) memset(stats, 0, sizeof *stats);
    hipStream_t s = (hipStream_t)stream;
    if (m == 0) {
        *total_weight_out = 0;
        if (stats) stats->base_cases = 1;
        return MSF_OK;
    }
    const size_t need = msf_workspace_bytes(m, n, opt);
    void* ws = workspace;
    bool owned = false;
    if (ws) {
        if (workspace_bytes < need) return MSF_EWORKSPACE;
        if ((uintptr_t)ws % 256) return MSF_EINVAL;   // its buffers take 16-byte vector accesses
    } else {
        if (hipMallocAsync(&ws, need, s) != hipSuccess) {
            (void)hipGetLastError();
            return MSF_ENOMEM;
        }
        owned = true;
    }
    Ctrl* hc = nullptr;
    st = take_pinned_ctrl(&hc);
    if (st == MSF_OK) {
        st = solve(u, v, w, m, n, mask_out, total_weight_out, (char*)ws, s, opt, stats, hc);
        give_pinned_ctrl(hc);
    }
    if (owned) {
        hipError_t e = hipFreeAsync(ws, s);
        hipError_t e2 = hipStreamSynchronize(s);
        if (st == MSF_OK && (e != hipSuccess || e2 != hipSuccess)) {
            set_err("hipFreeAsync", e != hipSuccess ? e : e2);
            st = MSF_EDEVICE;
        }
    }
    return st;
}

}  // extern "C"

// ------------------------------------------------------ no-allocation entry
// The workspace of msf_compute_noalloc: one array per GPU, held by the loaded
// library until the process ends.  On the host this name only stands for the
// symbol; the device address of each GPU's copy comes from
// hipGetSymbolAddress, and only that address is ever handed to kernels.
static __device__ __attribute__((aligned(256))) char scratch[MSF_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu[kScratchDevices];      // per GPU: set-up, then one call at a time
void* g_scratch_dev[kScratchDevices] = {};     // per GPU: device address of `scratch`
}  // namespace

extern "C" {

int msf_compute_noalloc(const int32_t* u, const int32_t* v, const uint32_t* w, int64_t m,
                        int64_t n, uint8_t* mask_out, uint64_t* total_weight_out, void* stream,
                        const msf_options* opt, msf_stats* stats) {
    int st = check_args(u, v, w, m, n, mask_out, total_weight_out, opt);
    if (st) return st;
    if (stats) memset(stats, 0, sizeof *stats);
    if (m == 0) {
        *total_weight_out = 0;
        if (stats) stats->base_cases = 1;
        return MSF_OK;
    }
    const size_t need = msf_workspace_bytes(m, n, opt);
    if (need > (size_t)MSF_NOALLOC_SCRATCH_BYTES) {
        char buf[160];
        snprintf(buf, sizeof buf,
                 "msf_compute_noalloc: the graph needs %zu workspace bytes, the static "
                 "scratch holds %zu",
                 need, (size_t)MSF_NOALLOC_SCRATCH_BYTES);
        set_err_text(buf);
        return MSF_EWORKSPACE;
    }
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kScratchDevices) {
        set_err_text("msf_compute_noalloc: device index beyond the scratch table");
        return MSF_EDEVICE;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu[dev]);
    if (!g_scratch_dev[dev]) {           // first call on this GPU, with it current
        void* p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        g_scratch_dev[dev] = p;
    }
    Ctrl hc;                              // ordinary host memory: nothing is allocated
    const bool prof_was_off = t_prof_off;
    t_prof_off = true;                    // the profiler would create events
    st = solve(u, v, w, m, n, mask_out, total_weight_out, (char*)g_scratch_dev[dev],
               (hipStream_t)stream, opt, stats, &hc);
    t_prof_off = prof_was_off;
    return st;
}

const char* msf_status_string(int status) {
    switch (status) {
        case MSF_OK: return "ok";
        case MSF_EINVAL: return "invalid argument";
        case MSF_ERANGE: return "vertex id out of range";
        case MSF_ENOMEM: return "device allocation failed";
        case MSF_EDEVICE: return "HIP runtime error";
        case MSF_EWORKSPACE: return "workspace too small";
        case MSF_EINTERNAL: return "internal error";
        default: return "unknown status";
    }
}

const char* msf_last_error(void) { return last_err(); }

int msf_version(void) { return 200; }

int msf_profile_enable(int on) {
    std::lock_guard<std::mutex> l(g_prof.mu);
    g_prof.on = on != 0;
    return MSF_OK;
}

int msf_profile_reset(void) {
    std::lock_guard<std::mutex> l(g_prof.mu);
    for (int k = 0; k < K_COUNT; ++k) {
        g_prof.launches[k] = 0;
        g_prof.ms[k] = 0;
        g_prof.bytes[k] = 0;
    }
    return MSF_OK;
}

int msf_profile_read(msf_kernel_profile* out, int capacity) {
    std::lock_guard<std::mutex> l(g_prof.mu);
    int n = 0;
    for (int k = 0; k < K_COUNT && n < capacity && out; ++k) {
        if (!g_prof.launches[k]) continue;
        memset(&out[n], 0, sizeof out[n]);
        strncpy(out[n].name, kKernelNames[k], sizeof out[n].name - 1);
        out[n].launches = g_prof.launches[k];
        out[n].total_ms = g_prof.ms[k];
        out[n].bytes = g_prof.bytes[k];
        ++n;
    }
    return n;
}

}  // extern "C"
