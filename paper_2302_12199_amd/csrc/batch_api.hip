// C ABI of the batched solver: argument checks, workspace carving, hipGraph
// capture and the autotuner.
#include <string.h>

#include "batch.h"
#include "host.h"

using namespace msf;

namespace {

constexpr int kTuneCoop[3] = {1 << 19, 1 << 20, -1};

struct Resolved {
    int block, lds_n, workgroups;
    int64_t coop_edges;
};

// Host-side defaults and checks (no device needed).
int resolve(const msf_batch_options* opt, Resolved* r) {
    r->block = 1024;
    r->lds_n = 2048;
    r->workgroups = 0;
    r->coop_edges = 1 << 20;
    if (opt) {
        for (int i = 0; i < 4; ++i)
            if (opt->reserved[i]) return MSF_EINVAL;
        if (opt->block) {
            if (opt->block != 256 && opt->block != 512 && opt->block != 1024) return MSF_EINVAL;
            r->block = opt->block;
        }
        if (opt->lds_vertices < -1 || opt->lds_vertices > 8192) return MSF_EINVAL;
        if (opt->lds_vertices == -1) r->lds_n = 0;
        else if (opt->lds_vertices > 0) r->lds_n = opt->lds_vertices;
        if (opt->workgroups < 0 || opt->workgroups > 65536) return MSF_EINVAL;
        r->workgroups = opt->workgroups;
        if (opt->coop_edges < -1) return MSF_EINVAL;
        if (opt->coop_edges == -1) r->coop_edges = -1;
        else if (opt->coop_edges > 0) r->coop_edges = opt->coop_edges;
    }
    return MSF_OK;
}

// Device-dependent part: the LDS limit and the default grid (as many
// workgroups as can be resident; nothing requires them all to be).
int fit_grid(Resolved* r) {
    if (!batch_allow_lds(r->block, (size_t)r->lds_n * 20)) r->lds_n = 64 * 1024 / 20;
    if (r->workgroups == 0) {
        r->workgroups = batch_resident_workgroups(r->block, (size_t)r->lds_n * 20);
        if (r->workgroups <= 0) {
            set_err_text("the batched kernel cannot be resident on this device");
            return MSF_EDEVICE;
        }
    }
    return MSF_OK;
}

int prepare(const int32_t* u, const int32_t* v, const uint32_t* w, const int64_t* eoff,
            const int64_t* voff, int64_t G, int64_t max_n, const int32_t* order, uint8_t* mask,
            uint64_t* totals, uint64_t* ticks, void* ws, size_t ws_bytes,
            const msf_batch_options* opt, BatchArgs* A, Resolved* r) {
    if (G < 0 || G > 0x7fffffffLL || max_n < 0 || max_n > 0x7fffffffLL) return MSF_EINVAL;
    int st = resolve(opt, r);
    if (st) return st;
    if (G == 0) return MSF_OK;
    if (!u || !v || !w || !eoff || !voff || !mask || !totals || !ws) return MSF_EINVAL;
    if ((uintptr_t)ws % 256) return MSF_EINVAL;   // its buffers take 16-byte vector accesses
    if (ws_bytes < batch_layout(G, max_n, 1).total) return MSF_EWORKSPACE;
    if ((st = fit_grid(r))) return st;
    const BatchLayout L = batch_layout(G, max_n, r->workgroups);
    if (ws_bytes < L.total) return MSF_EWORKSPACE;
    char* base = (char*)ws;
    A->u = u; A->v = v; A->w = w; A->eoff = eoff; A->voff = voff; A->G = G; A->order = order;
    A->mask = mask; A->totals = totals; A->ticks = ticks;
    A->q = (BatchQueue*)base;
    A->xw = (XcdWork*)(base + L.xw_off);
    A->big = (int32_t*)(base + L.lists_off);
    A->small = A->big + G;
    A->xslots = base + L.xslots_off;
    A->wslots = base + L.wslots_off;
    A->slot_bytes = batch_slot_bytes(max_n);
    A->xslot_bytes = batch_xslot_bytes(max_n);
    A->nmax = max_n;
    A->coop_edges = r->coop_edges;
    A->lds_n = r->lds_n;
    return MSF_OK;
}

}  // namespace

struct msf_batch_graph {
    hipGraph_t graph;
    hipGraphExec_t exec;
};

extern "C" {

size_t msf_batched_workspace_bytes(int64_t G, int64_t max_n, const msf_batch_options* opt) {
    if (G < 0 || max_n < 0) return 0;
    Resolved r;
    if (resolve(opt, &r) != MSF_OK) return 0;
    if (opt) {
        if (fit_grid(&r) != MSF_OK) return 0;
        return batch_layout(G, max_n, r.workgroups).total;
    }
    // large enough for the defaults and every autotuner candidate: the grid
    // is largest with the smallest block and LDS use
    msf_batch_options o;
    memset(&o, 0, sizeof o);
    o.block = 512;
    o.lds_vertices = 1024;
    Resolved rs;
    if (resolve(&o, &rs) != MSF_OK || fit_grid(&rs) != MSF_OK || fit_grid(&r) != MSF_OK) return 0;
    const int wg = rs.workgroups > r.workgroups ? rs.workgroups : r.workgroups;
    return batch_layout(G, max_n, wg).total;
}

int msf_compute_batched(const int32_t* u, const int32_t* v, const uint32_t* w,
                        const int64_t* edge_off, const int64_t* vert_off, int64_t G,
                        int64_t max_n, const int32_t* order, uint8_t* mask_out,
                        uint64_t* totals_out, uint64_t* ticks_out, void* workspace,
                        size_t workspace_bytes, void* stream, const msf_batch_options* opt) {
    BatchArgs A;
    Resolved r;
    int st = prepare(u, v, w, edge_off, vert_off, G, max_n, order, mask_out, totals_out,
                     ticks_out, workspace, workspace_bytes, opt, &A, &r);
    if (st || G == 0) return st;
    const int h = prof_begin(K_BATCH, (hipStream_t)stream);
    if (launch_batch(A, r.block, r.workgroups, (hipStream_t)stream) != 0) {
        set_err_text("batched launch failed");
        return MSF_EDEVICE;
    }
    prof_end(h, (hipStream_t)stream, 0.0);
    return MSF_OK;
}

int msf_batched_graph_create(const int32_t* u, const int32_t* v, const uint32_t* w,
                             const int64_t* edge_off, const int64_t* vert_off, int64_t G,
                             int64_t max_n, const int32_t* order, uint8_t* mask_out,
                             uint64_t* totals_out, uint64_t* ticks_out, void* workspace,
                             size_t workspace_bytes, const msf_batch_options* opt,
                             msf_batch_graph** graph_out) {
    if (!graph_out) return MSF_EINVAL;
    *graph_out = nullptr;
    BatchArgs A;
    Resolved r;
    int st = prepare(u, v, w, edge_off, vert_off, G, max_n, order, mask_out, totals_out,
                     ticks_out, workspace, workspace_bytes, opt, &A, &r);
    if (st) return st;
    hipStream_t cs;
    HIP_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    msf_batch_graph* g = new msf_batch_graph();
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        if (G > 0) launch_batch(A, r.block, r.workgroups, cs);
        e = hipStreamEndCapture(cs, &g->graph);
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
    (void)hipStreamDestroy(cs);
    if (e != hipSuccess) {
        set_err("graph capture", e);
        delete g;
        return MSF_EDEVICE;
    }
    *graph_out = g;
    return MSF_OK;
}

int msf_batched_graph_launch(msf_batch_graph* graph, void* stream) {
    if (!graph) return MSF_EINVAL;
    HIP_TRY(hipGraphLaunch(graph->exec, (hipStream_t)stream));
    return MSF_OK;
}

int msf_batched_graph_destroy(msf_batch_graph* graph) {
    if (!graph) return MSF_EINVAL;
    (void)hipGraphExecDestroy(graph->exec);
    (void)hipGraphDestroy(graph->graph);
    delete graph;
    return MSF_OK;
}

int msf_batched_autotune(const int32_t* u, const int32_t* v, const uint32_t* w,
                         const int64_t* edge_off, const int64_t* vert_off, int64_t G,
                         int64_t max_n, const int32_t* order, uint8_t* mask_out,
                         uint64_t* totals_out, void* workspace, size_t workspace_bytes,
                         void* stream, msf_batch_options* best_out, float* best_ms_out) {
    if (!best_out) return MSF_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const int blocks[2] = {512, 1024};
    const int ldss[3] = {1024, 2048, 4096};
    hipEvent_t a, b;
    HIP_TRY(hipEventCreate(&a));
    HIP_TRY(hipEventCreate(&b));
    float best_ms = -1.f;
    msf_batch_options best;
    memset(&best, 0, sizeof best);
    for (int bi = 0; bi < 2; ++bi) {
        for (int li = 0; li < 3; ++li) {
            for (int coop : kTuneCoop) {
                msf_batch_options o;
                memset(&o, 0, sizeof o);
                o.block = blocks[bi];
                o.lds_vertices = ldss[li];
                o.coop_edges = coop;
                float ms = 0.f;
                for (int rep = 0; rep < 2; ++rep) {   // first run warms up
                    HIP_TRY(hipEventRecord(a, s));
                    int st = msf_compute_batched(u, v, w, edge_off, vert_off, G, max_n, order,
                                                 mask_out, totals_out, nullptr, workspace,
                                                 workspace_bytes, stream, &o);
                    if (st == MSF_EWORKSPACE) break;   // candidate needs more workspace
                    if (st) { (void)hipEventDestroy(a); (void)hipEventDestroy(b); return st; }
                    HIP_TRY(hipEventRecord(b, s));
                    HIP_TRY(hipEventSynchronize(b));
                    HIP_TRY(hipEventElapsedTime(&ms, a, b));
                }
                if (ms > 0.f && (best_ms < 0.f || ms < best_ms)) { best_ms = ms; best = o; }
            }
        }
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (best_ms < 0.f) return MSF_EWORKSPACE;
    *best_out = best;
    if (best_ms_out) *best_ms_out = best_ms;
    return MSF_OK;
}

int msf_wall_clock_khz(void) {
    int dev = 0, khz = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return khz;
}

}  // extern "C"
