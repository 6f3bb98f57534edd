// Borůvka round kernels (paper Sec. II-C; Alg. 1 round body of Sec. IV).
//
// One round on the edge list of the current graph:
//   minedge      best[x] = min key over live edges incident to x   (minEdges)
//   hook         parent[x] = other endpoint of best[x]; the smaller vertex of
//                each 2-cycle becomes the root; every non-root marks its edge
//                as an MSF edge                                     (contractComponents)
//   jump         parent[x] <- parent[parent[x]] until stars         (pointer doubling)
//   scan_roots   dense new ids for roots that still have edges      (base-case style relabel)
//   label        label[x] = new id of x's root
//   relabel      (label[u], label[v]), drop self-loops, stable compaction, fused
//                with the next round's minedge                       (relabel)
// Keys are (w << 32 | position) with positions in edge-id order, so every
// comparison is the paper's consistent tie break by (weight, edge id).
#include "prim.h"

namespace msf {

__global__ void k_fill_u64(uint64_t* __restrict__ p, int64_t n, uint64_t val) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = val;
}

__global__ void k_zero_bytes(uint8_t* __restrict__ p, int64_t n) {
    const int64_t nv = n >> 4;
    uint4* q = reinterpret_cast<uint4*>(p);
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nv;
         i += (int64_t)gridDim.x * blockDim.x)
        q[i] = make_uint4(0, 0, 0, 0);
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t < (n & 15)) p[(nv << 4) + t] = 0;
}

// Clears a lookback status array and the tile counter before a scan launch,
// and the per-round counters when `round_begin` is set.
__global__ void k_scan_prep(uint64_t* __restrict__ status, int64_t ntiles, Ctrl* ctrl,
                            int round_begin) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < ntiles;
         i += (int64_t)gridDim.x * blockDim.x)
        status[i] = 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        ctrl->tile_counter = 0;
        if (round_begin) {
            ctrl->live = 0;
            ctrl->found = 0;
            ctrl->jump_more = 0;
        }
    }
}

// Round 0 lightest incident edge, reading the caller's arrays directly.
// Validates ids (bit kErrRange) and skips self-loops.
__global__ __launch_bounds__(kBlock) void k_minedge_r0(
    const int32_t* __restrict__ u, const int32_t* __restrict__ v, const uint32_t* __restrict__ w,
    int64_t m, int64_t n, uint64_t* __restrict__ best, Ctrl* ctrl) {
    bool bad = false;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < m;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int32_t a = u[e], b = v[e];
        if ((uint32_t)a >= (uint64_t)n || (uint32_t)b >= (uint64_t)n) { bad = true; continue; }
        if (a == b) continue;
        const uint64_t key = ((uint64_t)w[e] << 32) | (uint64_t)e;
        atomic_min_key(&best[a], key);
        atomic_min_key(&best[b], key);
    }
    if (__ballot(bad) && lane_id() == 0) atomicOr(&ctrl->err, kErrRange);
}

// Hook: parent[x] = other endpoint of x's lightest edge.  Both vertices of a
// 2-cycle picked the same edge (strict order), recognised as best[other] ==
// best[x]; the smaller id is the root.  Every other live vertex owns exactly
// one MSF edge and marks it, so each MSF edge is counted once.
template <bool kR0>
__global__ __launch_bounds__(kBlock) void k_hook(
    const uint64_t* __restrict__ best, int64_t nr, const int32_t* __restrict__ U,
    const int32_t* __restrict__ V, const uint32_t* __restrict__ ID, int32_t* __restrict__ parent,
    uint8_t* __restrict__ mask, Ctrl* ctrl) {
    uint64_t wsum = 0, nfound = 0, nlive = 0;
    bool bad = false;
    for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < nr;
         x += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t b = best[x];
        if (b == kKeyMax) { parent[x] = (int32_t)x; continue; }
        ++nlive;
        const uint32_t pos = (uint32_t)b;
        const int32_t eu = U[pos], ev = V[pos];
        if (eu != x && ev != x) bad = true;
        const int32_t other = eu == (int32_t)x ? ev : eu;
        if (best[other] == b && (int32_t)x < other) {
            parent[x] = (int32_t)x;
        } else {
            parent[x] = other;
            const uint32_t id = kR0 ? pos : ID[pos];
            mask[id] = 1;
            wsum += b >> 32;
            ++nfound;
        }
    }
    wsum = wave_sum_u64(wsum);
    nfound = wave_sum_u64(nfound);
    nlive = wave_sum_u64(nlive);
    if (lane_id() == 0) {
        if (nfound) {
            atomicAdd((unsigned long long*)&ctrl->total, (unsigned long long)wsum);
            atomicAdd((unsigned long long*)&ctrl->msf_edges, (unsigned long long)nfound);
            atomicAdd((unsigned long long*)&ctrl->found, (unsigned long long)nfound);
        }
        if (nlive) atomicAdd((unsigned long long*)&ctrl->live, (unsigned long long)nlive);
    }
    if (__ballot(bad) && lane_id() == 0) atomicOr(&ctrl->err, kErrInternal);
}

// Pointer jumping in place: each vertex repeatedly replaces its parent by its
// grandparent.  Values only ever move towards the root, so reading a stale or
// concurrently updated entry is harmless.  At most `iters` steps per launch;
// a vertex that has not reached its root raises jump_more.
__global__ __launch_bounds__(kBlock) void k_jump(int32_t* __restrict__ parent, int64_t nr,
                                                 int iters, Ctrl* ctrl) {
    bool more = false;
    for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < nr;
         x += (int64_t)gridDim.x * blockDim.x) {
        int32_t p = parent[x];
        if (p == (int32_t)x) continue;
        int32_t pp = parent[p];
        int it = 0;
        while (pp != p && it < iters) {
            p = pp;
            parent[x] = p;
            pp = parent[p];
            ++it;
        }
        if (pp != p) more = true;
    }
    if (__ballot(more) && lane_id() == 0) ctrl->jump_more = 1;
}

// Dense ids for the roots that still have edges: stable scan over the flags
// (parent[x] == x && best[x] != MAX); root x gets label[x] = its rank.
__global__ __launch_bounds__(kBlock) void k_scan_roots(
    const int32_t* __restrict__ parent, const uint64_t* __restrict__ best, int64_t nr,
    int32_t* __restrict__ label, uint64_t* status, Ctrl* ctrl, uint32_t ntiles) {
    __shared__ uint32_t s_tile;
    __shared__ uint32_t s_wave[kBlock / kWave];
    __shared__ uint64_t s_prefix;
    const uint32_t tile = take_tile(ctrl, &s_tile);
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int64_t wbase = (int64_t)tile * kTile + (int64_t)wave * (kWave * kItems);
    uint64_t mk[kItems];
    uint32_t cnt = 0;
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        const int64_t x = wbase + k * kWave + lane;
        bool f = false;
        if (x < nr) f = parent[x] == (int32_t)x && best[x] != kKeyMax;
        mk[k] = __ballot(f);
        cnt += __popcll(mk[k]);
    }
    if (lane == 0) s_wave[wave] = cnt;
    __syncthreads();
    uint32_t agg = 0, woff = 0;
#pragma unroll
    for (int i = 0; i < kBlock / kWave; ++i) {
        if (i < wave) woff += s_wave[i];
        agg += s_wave[i];
    }
    const uint64_t prefix = tile_prefix(status, tile, agg, ctrl, &s_prefix);
    uint64_t off = prefix + woff;
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        const int64_t x = wbase + k * kWave + lane;
        if ((mk[k] >> lane) & 1) label[x] = (int32_t)(off + lanes_below(mk[k]));
        off += __popcll(mk[k]);
    }
    if (tile == ntiles - 1 && threadIdx.x == 0) ctrl->n_next = prefix + agg;
}

// label[x] for non-roots from their root; -1 for vertices without edges.
// Also resets best_next[0, n_next) for the fused next-round minedge.
__global__ __launch_bounds__(kBlock) void k_label(
    const int32_t* __restrict__ parent, const uint64_t* __restrict__ best, int64_t nr,
    int32_t* __restrict__ label, uint64_t* __restrict__ best_next, const Ctrl* ctrl) {
    const int64_t nn = (int64_t)ctrl->n_next;
    for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < nr;
         x += (int64_t)gridDim.x * blockDim.x) {
        const int32_t p = parent[x];
        if (best[x] == kKeyMax) label[x] = -1;
        else if (p != (int32_t)x) label[x] = label[p];
        if (x < nn) best_next[x] = kKeyMax;
    }
}

// Relabel every edge to (label[u], label[v]), drop the self-loops this
// creates, and compact the survivors stably into `out` (position order stays
// edge-id order).  Fused: each survivor immediately takes part in the next
// round's lightest-edge search with key (w << 32 | new position).
template <bool kR0>
__global__ __launch_bounds__(kBlock) void k_relabel(
    const int32_t* __restrict__ U, const int32_t* __restrict__ V, const uint32_t* __restrict__ W,
    const uint32_t* __restrict__ ID, int64_t mr, const int32_t* __restrict__ label, EdgeSoA out,
    uint64_t* __restrict__ best_next, uint64_t* status, Ctrl* ctrl, uint32_t ntiles) {
    constexpr int kIt = kRelabelItems;
    __shared__ uint32_t s_tile;
    __shared__ uint32_t s_wave[kBlock / kWave];
    __shared__ uint64_t s_prefix;
    const uint32_t tile = take_tile(ctrl, &s_tile);
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int64_t e0 = (int64_t)tile * (kBlock * kIt) + (int64_t)wave * (kWave * kIt) + lane;
    int32_t a[kIt], b[kIt];
    uint64_t mk[kIt];
    uint32_t cnt = 0;
#pragma unroll
    for (int k = 0; k < kIt; ++k) {
        const int64_t e = e0 + k * kWave;
        a[k] = b[k] = 0;
        if (e < mr) { a[k] = U[e]; b[k] = V[e]; }
    }
#pragma unroll
    for (int k = 0; k < kIt; ++k) {
        const int64_t e = e0 + k * kWave;
        bool keep = false;
        if (e < mr) {
            a[k] = label[a[k]];
            b[k] = label[b[k]];
            keep = a[k] != b[k];
        }
        mk[k] = __ballot(keep);
        cnt += __popcll(mk[k]);
    }
    if (lane == 0) s_wave[wave] = cnt;
    __syncthreads();
    uint32_t agg = 0, woff = 0;
#pragma unroll
    for (int i = 0; i < kBlock / kWave; ++i) {
        if (i < wave) woff += s_wave[i];
        agg += s_wave[i];
    }
    const uint64_t prefix = tile_prefix(status, tile, agg, ctrl, &s_prefix);
    uint64_t off = prefix + woff;
#pragma unroll
    for (int k = 0; k < kIt; ++k) {
        const int64_t e = e0 + k * kWave;
        if ((mk[k] >> lane) & 1) {
            const uint64_t o = off + lanes_below(mk[k]);
            const uint32_t wt = W[e];
            out.u[o] = a[k];
            out.v[o] = b[k];
            out.w[o] = wt;
            out.id[o] = kR0 ? (uint32_t)e : ID[e];
            const uint64_t key = ((uint64_t)wt << 32) | o;
            atomic_min_key(&best_next[a[k]], key);
            atomic_min_key(&best_next[b[k]], key);
        }
        off += __popcll(mk[k]);
    }
    if (tile == ntiles - 1 && threadIdx.x == 0) ctrl->m_next = prefix + agg;
}

// ------------------------------------------------------------------ launchers

static inline unsigned grid_for(int64_t n, unsigned cap = 2048) {
    int64_t g = (n + kBlock - 1) / kBlock;
    if (g < 1) g = 1;
    return (unsigned)(g < cap ? g : cap);
}

void launch_fill_u64(uint64_t* p, int64_t n, uint64_t val, hipStream_t s) {
    if (n > 0) hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(n)), dim3(kBlock), 0, s, p, n, val);
}
void launch_zero_bytes(uint8_t* p, int64_t n, hipStream_t s) {
    if (n > 0)
        hipLaunchKernelGGL(k_zero_bytes, dim3(grid_for((n >> 4) + 16)), dim3(kBlock), 0, s, p, n);
}
void launch_scan_prep(uint64_t* status, int64_t ntiles, Ctrl* ctrl, int round_begin,
                      hipStream_t s) {
    hipLaunchKernelGGL(k_scan_prep, dim3(grid_for(ntiles, 256)), dim3(kBlock), 0, s, status,
                       ntiles, ctrl, round_begin);
}
void launch_minedge_r0(const int32_t* u, const int32_t* v, const uint32_t* w, int64_t m,
                       int64_t n, uint64_t* best, Ctrl* ctrl, hipStream_t s) {
    if (m > 0)
        hipLaunchKernelGGL(k_minedge_r0, dim3(grid_for(m)), dim3(kBlock), 0, s, u, v, w, m, n,
                           best, ctrl);
}
void launch_hook(bool r0, const uint64_t* best, int64_t nr, const int32_t* U, const int32_t* V,
                 const uint32_t* ID, int32_t* parent, uint8_t* mask, Ctrl* ctrl, hipStream_t s) {
    if (r0)
        hipLaunchKernelGGL(k_hook<true>, dim3(grid_for(nr)), dim3(kBlock), 0, s, best, nr, U, V,
                           ID, parent, mask, ctrl);
    else
        hipLaunchKernelGGL(k_hook<false>, dim3(grid_for(nr)), dim3(kBlock), 0, s, best, nr, U,
                           V, ID, parent, mask, ctrl);
}
void launch_jump(int32_t* parent, int64_t nr, int iters, Ctrl* ctrl, hipStream_t s) {
    hipLaunchKernelGGL(k_jump, dim3(grid_for(nr)), dim3(kBlock), 0, s, parent, nr, iters, ctrl);
}
void launch_scan_roots(const int32_t* parent, const uint64_t* best, int64_t nr, int32_t* label,
                       uint64_t* status, Ctrl* ctrl, hipStream_t s) {
    const uint32_t nt = (uint32_t)((nr + kTile - 1) / kTile);
    hipLaunchKernelGGL(k_scan_roots, dim3(nt), dim3(kBlock), 0, s, parent, best, nr, label,
                       status, ctrl, nt);
}
void launch_label(const int32_t* parent, const uint64_t* best, int64_t nr, int32_t* label,
                  uint64_t* best_next, const Ctrl* ctrl, hipStream_t s) {
    hipLaunchKernelGGL(k_label, dim3(grid_for(nr)), dim3(kBlock), 0, s, parent, best, nr, label,
                       best_next, ctrl);
}
void launch_relabel(bool r0, const int32_t* U, const int32_t* V, const uint32_t* W,
                    const uint32_t* ID, int64_t mr, const int32_t* label, EdgeSoA out,
                    uint64_t* best_next, uint64_t* status, Ctrl* ctrl, hipStream_t s) {
    const uint32_t nt = (uint32_t)((mr + kRelabelTile - 1) / kRelabelTile);
    if (r0)
        hipLaunchKernelGGL(k_relabel<true>, dim3(nt), dim3(kBlock), 0, s, U, V, W, ID, mr, label,
                           out, best_next, status, ctrl, nt);
    else
        hipLaunchKernelGGL(k_relabel<false>, dim3(nt), dim3(kBlock), 0, s, U, V, W, ID, mr,
                           label, out, best_next, status, ctrl, nt);
}

}  // namespace msf
