// C ABI of the MSF library: argument checks, workspace carving and the
// host-side round driver.  Every step of the computation runs in the HIP
// kernels; the host only sizes launches from two counters read back per round.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "../../include/msf.h"
#include "common.h"

namespace msf {
void launch_fill_u64(uint64_t* p, int64_t n, uint64_t val, hipStream_t s);
void launch_zero_bytes(uint8_t* p, int64_t n, hipStream_t s);
void launch_scan_prep(uint64_t* status, int64_t ntiles, Ctrl* ctrl, int round_begin,
                      hipStream_t s);
void launch_minedge_r0(const int32_t* u, const int32_t* v, const uint32_t* w, int64_t m,
                       int64_t n, uint64_t* best, Ctrl* ctrl, hipStream_t s);
void launch_hook(bool r0, const uint64_t* best, int64_t nr, const int32_t* U, const int32_t* V,
                 const uint32_t* ID, int32_t* parent, uint8_t* mask, Ctrl* ctrl, hipStream_t s);
void launch_jump(int32_t* parent, int64_t nr, int iters, Ctrl* ctrl, hipStream_t s);
void launch_scan_roots(const int32_t* parent, const uint64_t* best, int64_t nr, int32_t* label,
                       uint64_t* status, Ctrl* ctrl, hipStream_t s);
void launch_label(const int32_t* parent, const uint64_t* best, int64_t nr, int32_t* label,
                  uint64_t* best_next, const Ctrl* ctrl, hipStream_t s);
void launch_relabel(bool r0, const int32_t* U, const int32_t* V, const uint32_t* W,
                    const uint32_t* ID, int64_t mr, const int32_t* label, EdgeSoA out,
                    uint64_t* best_next, uint64_t* status, Ctrl* ctrl, hipStream_t s);
}  // namespace msf

using namespace msf;

namespace {

thread_local char g_err[512];

void set_err(const char* what, hipError_t e) {
    snprintf(g_err, sizeof g_err, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_TRY(call)                                   \
    do {                                                \
        hipError_t e_ = (call);                         \
        if (e_ != hipSuccess) {                         \
            set_err(#call, e_);                         \
            return MSF_EDEVICE;                         \
        }                                               \
    } while (0)

// ------------------------------------------------------------ kernel timing
enum KernelId { K_MINEDGE_R0, K_HOOK, K_JUMP, K_SCAN_ROOTS, K_LABEL, K_RELABEL, K_FILL,
                K_PREP, K_COUNT };
const char* const kKernelNames[K_COUNT] = {"minedge_r0", "hook", "jump", "scan_roots",
                                           "label", "relabel", "fill", "scan_prep"};

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

bool prof_on() {
    std::lock_guard<std::mutex> l(g_prof.mu);
    return g_prof.on;
}

// Starts timing one launch of kernel `kid`; returns a handle (or -1 when off).
int prof_begin(int kid, hipStream_t s) {
    std::lock_guard<std::mutex> l(g_prof.mu);
    if (!g_prof.on) return -1;
    std::pair<hipEvent_t, hipEvent_t> ev;
    if (!g_prof.pool.empty()) {
        ev = g_prof.pool.back();
        g_prof.pool.pop_back();
    } else if (hipEventCreate(&ev.first) != hipSuccess || hipEventCreate(&ev.second) != hipSuccess) {
        return -1;
    }
    (void)hipEventRecord(ev.first, s);
    g_prof.pending.push_back({kid, ev.first, ev.second, 0.0});
    return (int)g_prof.pending.size() - 1;
}

void prof_end(int h, hipStream_t s, double bytes) {
    if (h < 0) return;
    std::lock_guard<std::mutex> l(g_prof.mu);
    (void)hipEventRecord(g_prof.pending[h].b, s);
    g_prof.pending[h].bytes += bytes;
}

void prof_add_bytes(int h, double bytes) {
    if (h < 0) return;
    std::lock_guard<std::mutex> l(g_prof.mu);
    g_prof.pending[h].bytes += bytes;
}

// Accumulates every pending launch; call only after the stream is synchronised.
void prof_resolve() {
    std::lock_guard<std::mutex> l(g_prof.mu);
    for (auto& p : g_prof.pending) {
        float t = 0.f;
        if (hipEventElapsedTime(&t, p.a, p.b) == hipSuccess) {
            g_prof.launches[p.kid] += 1;
            g_prof.ms[p.kid] += t;
            g_prof.bytes[p.kid] += p.bytes;
        }
        g_prof.pool.push_back({p.a, p.b});
    }
    g_prof.pending.clear();
}

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Workspace layout for plain Borůvka on (m, n).
struct Layout {
    size_t ctrl, best0, best1, parent, label, status, ea[4], eb[4], total;
};

Layout layout(int64_t m, int64_t n) {
    Layout L;
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off += align_up(bytes ? bytes : 1); return o; };
    const size_t nn = (size_t)(n > 0 ? n : 1), mm = (size_t)(m > 0 ? m : 1);
    const int64_t tile_min = kTile < kRelabelTile ? kTile : kRelabelTile;
    const size_t tiles = (size_t)((std::max<int64_t>(m, n) + tile_min - 1) / tile_min) + 1;
    L.ctrl = take(sizeof(Ctrl));
    L.status = take(tiles * 8);
    L.best0 = take(nn * 8);
    L.best1 = take(nn * 8);
    L.parent = take(nn * 4);
    L.label = take(nn * 4);
    for (int i = 0; i < 4; ++i) L.ea[i] = take(mm * 4);
    for (int i = 0; i < 4; ++i) L.eb[i] = take(mm * 4);
    L.total = off;
    return L;
}

// Small pinned host buffer for the per-round counter read-back.
struct HostCtrl {
    std::mutex mu;
    Ctrl* p = nullptr;
};
HostCtrl g_host;

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
        if (opt->sample_size < 0 || opt->sample_size > (1 << 16)) return MSF_EINVAL;
        if (opt->sparse_degree < 0 || opt->min_split_edges < 0) return MSF_EINVAL;
        for (int i = 0; i < 8; ++i)
            if (opt->reserved[i]) return MSF_EINVAL;
    }
    return MSF_OK;
}

int read_ctrl(Ctrl* dctrl, Ctrl* host, hipStream_t s) {
    HIP_TRY(hipMemcpyAsync(host, dctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    prof_resolve();
    return MSF_OK;
}

// Plain Borůvka on the caller's arrays with a carved workspace.
int boruvka_solve(const int32_t* u, const int32_t* v, const uint32_t* w, int64_t m, int64_t n,
                  uint8_t* mask, uint64_t* total_out, char* ws, hipStream_t s,
                  msf_stats* stats) {
    const Layout L = layout(m, n);
    Ctrl* dctrl = (Ctrl*)(ws + L.ctrl);
    uint64_t* status = (uint64_t*)(ws + L.status);
    uint64_t* best_cur = (uint64_t*)(ws + L.best0);
    uint64_t* best_nxt = (uint64_t*)(ws + L.best1);
    int32_t* parent = (int32_t*)(ws + L.parent);
    int32_t* label = (int32_t*)(ws + L.label);
    EdgeSoA bufA = {(int32_t*)(ws + L.ea[0]), (int32_t*)(ws + L.ea[1]),
                    (uint32_t*)(ws + L.ea[2]), (uint32_t*)(ws + L.ea[3])};
    EdgeSoA bufB = {(int32_t*)(ws + L.eb[0]), (int32_t*)(ws + L.eb[1]),
                    (uint32_t*)(ws + L.eb[2]), (uint32_t*)(ws + L.eb[3])};

    std::lock_guard<std::mutex> lock(g_host.mu);
    if (!g_host.p) HIP_TRY(hipHostMalloc((void**)&g_host.p, sizeof(Ctrl), hipHostMallocDefault));
    Ctrl* hc = g_host.p;

    HIP_TRY(hipMemsetAsync(dctrl, 0, sizeof(Ctrl), s));
    int h = prof_begin(K_FILL, s);
    launch_zero_bytes(mask, m, s);
    launch_fill_u64(best_cur, n, kKeyMax, s);
    prof_end(h, s, (double)m + 8.0 * n);
    h = prof_begin(K_MINEDGE_R0, s);
    launch_minedge_r0(u, v, w, m, n, best_cur, dctrl, s);
    prof_end(h, s, 12.0 * m + 8.0 * n);
    HIP_TRY(hipGetLastError());
    int st = read_ctrl(dctrl, hc, s);
    if (st) return st;
    if (hc->err & kErrRange) return MSF_ERANGE;

    int64_t nr = n, mr = m;
    bool r0 = true;
    const int32_t *U = u, *V = v;
    const uint32_t *W = w, *ID = nullptr;
    EdgeSoA out = bufA, spare = bufB;
    uint32_t rounds = 0;
    while (mr > 0) {
        launch_scan_prep(status, 0, dctrl, 1, s);
        const int hh = prof_begin(K_HOOK, s);
        launch_hook(r0, best_cur, nr, U, V, ID, parent, mask, dctrl, s);
        prof_end(hh, s, 12.0 * nr);
        h = prof_begin(K_JUMP, s);
        launch_jump(parent, nr, 32, dctrl, s);
        prof_end(h, s, 12.0 * nr);
        HIP_TRY(hipGetLastError());
        if ((st = read_ctrl(dctrl, hc, s))) return st;
        const uint64_t live = hc->live, found = hc->found;
        prof_add_bytes(hh, 17.0 * live);  // per live vertex: edge endpoints, best[other], mask
        for (int pass = 0; hc->jump_more; ++pass) {
            if (pass > 64) {
                snprintf(g_err, sizeof g_err, "pointer jumping did not converge");
                return MSF_EINTERNAL;
            }
            HIP_TRY(hipMemsetAsync(&dctrl->jump_more, 0, sizeof(uint32_t), s));
            h = prof_begin(K_JUMP, s);
            launch_jump(parent, nr, 32, dctrl, s);
            prof_end(h, s, 12.0 * nr);
            HIP_TRY(hipGetLastError());
            if ((st = read_ctrl(dctrl, hc, s))) return st;
        }
        const int64_t ntv = (nr + kTile - 1) / kTile;
        launch_scan_prep(status, ntv, dctrl, 0, s);
        const int hs = prof_begin(K_SCAN_ROOTS, s);
        launch_scan_roots(parent, best_cur, nr, label, status, dctrl, s);
        prof_end(hs, s, 12.0 * nr);
        const int hl = prof_begin(K_LABEL, s);
        launch_label(parent, best_cur, nr, label, best_nxt, dctrl, s);
        prof_end(hl, s, 16.0 * nr);
        const int64_t nte = (mr + kRelabelTile - 1) / kRelabelTile;
        launch_scan_prep(status, nte, dctrl, 0, s);
        const int hr = prof_begin(K_RELABEL, s);
        launch_relabel(r0, U, V, W, ID, mr, label, out, best_nxt, status, dctrl, s);
        prof_end(hr, s, (r0 ? 12.0 : 16.0) * mr + 8.0 * mr);
        HIP_TRY(hipGetLastError());
        // survivors' bytes are known once the counters are back
        if ((st = read_ctrl(dctrl, hc, s))) return st;
        if (prof_on()) {
            // fold the data-dependent parts into the totals just resolved
            std::lock_guard<std::mutex> l(g_prof.mu);
            g_prof.bytes[K_RELABEL] += 16.0 * hc->m_next + 8.0 * hc->n_next;
            g_prof.bytes[K_SCAN_ROOTS] += 4.0 * hc->n_next;
            g_prof.bytes[K_LABEL] += 8.0 * hc->n_next;
        }
        if (hc->err) {
            snprintf(g_err, sizeof g_err, "device error bits 0x%x in round %u", hc->err, rounds);
            return MSF_EINTERNAL;
        }
        if (stats && rounds < MSF_MAX_TRACE) {
            stats->round_live[rounds] = live;
            stats->round_edges[rounds] = (uint64_t)(r0 ? m : mr);
            stats->round_found[rounds] = found;
        }
        ++rounds;
        nr = (int64_t)hc->n_next;
        mr = (int64_t)hc->m_next;
        U = out.u; V = out.v; W = out.w; ID = out.id;
        std::swap(best_cur, best_nxt);
        std::swap(out, spare);
        r0 = false;
        if (rounds > 70) { snprintf(g_err, sizeof g_err, "too many rounds"); return MSF_EINTERNAL; }
    }
    if ((st = read_ctrl(dctrl, hc, s))) return st;
    *total_out = hc->total;
    if (stats) {
        stats->total_weight = hc->total;
        stats->msf_edges = hc->msf_edges;
        stats->rounds = rounds;
        stats->base_cases = 1;
    }
    return MSF_OK;
}

}  // namespace

extern "C" {

size_t msf_workspace_bytes(int64_t m, int64_t n, const msf_options* opt) {
    (void)opt;
    if (m < 0 || n < 0) return 0;
    return layout(m, n).total;
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
    } else {
        const char* fail = getenv("MSF_TEST_FAIL_ALLOC");
        if (fail && fail[0] == '1') return MSF_ENOMEM;
        if (hipMallocAsync(&ws, need, s) != hipSuccess) {
            (void)hipGetLastError();
            return MSF_ENOMEM;
        }
        owned = true;
    }
    st = boruvka_solve(u, v, w, m, n, mask_out, total_weight_out, (char*)ws, s, stats);
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

const char* msf_last_error(void) { return g_err; }

int msf_version(void) { return 100; }

int msf_profile_enable(int on) {
    std::lock_guard<std::mutex> l(g_prof.mu);
    g_prof.on = on != 0;
    return MSF_OK;
}

int msf_profile_reset(void) {
    std::lock_guard<std::mutex> l(g_prof.mu);
    for (int k = 0; k < K_COUNT; ++k) { g_prof.launches[k] = 0; g_prof.ms[k] = 0; g_prof.bytes[k] = 0; }
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
