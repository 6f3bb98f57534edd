// Borůvka round kernels (paper Sec. II-C; the round body of Alg. 1, Sec. IV).
//
// One round on the current graph:
//   minedge      best[x] = min key over live edges incident to x   (minEdges;
//                packed (w << 32 | position) keys, 64-bit atomicMin)
//   hook         parent[x] = other endpoint of best[x]; the smaller vertex of
//                each 2-cycle becomes the root; every non-root marks its edge
//                as an MSF edge                                     (contractComponents)
//   jump         parent[x] <- parent[parent[x]] until stars         (pointer doubling)
//   scan_roots   dense new ids for roots that still have edges      (dense relabel of the base case)
//   label        label[x] = new id of x's root
//   pass         every edge is relabelled through the label map, self-loops
//                are dropped, and the survivors immediately take part in the
//                next round's minedge (relabel fused with minEdges)
// The pass either keeps the edge positions (rewriting endpoint labels, or
// only composing the label map when nothing needs rewriting) or compacts the
// live edges stably (keep bits and counts per tile, a scan of the counts, a
// scatter).
#include <stdlib.h>

#include <atomic>

#include "launch.h"
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

// Clears a lookback status array and the tile counter before a scan launch.
// round_begin also clears the per-round counters.
__global__ void k_scan_prep(uint64_t* __restrict__ status, int64_t ntiles, Ctrl* ctrl,
                            int round_begin) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < ntiles;
         i += (int64_t)gridDim.x * blockDim.x)
        status[i] = 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        ctrl->tile_counter = 0;
        if (round_begin) {   // m_next stays: the last pass's count is read with this round's
            ctrl->live = 0;
            ctrl->found = 0;
            ctrl->jump_more = 0;
        }
    }
}

// ------------------------------------------------------------ edge access

template <int MODE>
__device__ __forceinline__ void load_ends(const View& g, int64_t p, int32_t& a, int32_t& b) {
    if constexpr (MODE == kFull16) {
        const uint32_t x = g.p16[p];
        a = (int32_t)(x & 0xffffu);
        b = (int32_t)(x >> 16);
    } else {
        a = g.u[p];
        b = g.v[p];
    }
}

template <int MODE>
__device__ __forceinline__ uint32_t edge_id(const View& g, int64_t p) {
    if constexpr (MODE == kCompact) return g.id[p];
    else return (uint32_t)p;
}

// ---------------------------------------------------------------- round 0

// Lightest incident edge on the caller's arrays (4 edges per lane when the
// arrays are 16-byte aligned).  Validates ids (kErrRange), skips self-loops.
// `hot` (or -1) names a vertex expected on very many edges (the largest
// component after a filter step): its minimum is taken in LDS per workgroup
// and merged with one global atomic at the end.  sh = 1: side keys, w << 32
// | position << 1 | side (side 1 at the v end; m <= 2^31); sh = 0: w << 32 |
// position.
template <int VEC>
__global__ __launch_bounds__(kBlock) void k_minedge_r0(
    const int32_t* __restrict__ u, const int32_t* __restrict__ v, const uint32_t* __restrict__ w,
    int64_t m, int64_t n, uint64_t* __restrict__ best, Ctrl* ctrl, int32_t hot, int sh) {
    __shared__ unsigned long long s_hot;
    if (threadIdx.x == 0) s_hot = kKeyMax;
    __syncthreads();
    bool bad = false;
    const int64_t groups = (m + VEC - 1) / VEC;
    // the loop bound is uniform over the workgroup: every wave runs each step
    // with all lanes (wave_min_update needs whole waves)
    for (int64_t g0 = blockIdx.x * (int64_t)blockDim.x; g0 < groups;
         g0 += (int64_t)gridDim.x * blockDim.x) {
        const int64_t g = g0 + threadIdx.x;
        int32_t aa[VEC], bb[VEC];
        uint32_t ww[VEC];
        if (VEC == 4 && g * 4 + 3 < m) {
            const int4 a4 = reinterpret_cast<const int4*>(u)[g];
            const int4 b4 = reinterpret_cast<const int4*>(v)[g];
            const uint4 w4 = reinterpret_cast<const uint4*>(w)[g];
            aa[0] = a4.x; aa[1] = a4.y; aa[2] = a4.z; aa[3] = a4.w;
            bb[0] = b4.x; bb[1] = b4.y; bb[2] = b4.z; bb[3] = b4.w;
            ww[0] = w4.x; ww[1] = w4.y; ww[2] = w4.z; ww[3] = w4.w;
        } else {
#pragma unroll
            for (int k = 0; k < VEC; ++k) {
                const int64_t e = g * VEC + k;
                aa[k] = bb[k] = 0;
                ww[k] = 0;
                if (e < m) { aa[k] = u[e]; bb[k] = v[e]; ww[k] = w[e]; }
            }
        }
#pragma unroll
        for (int k = 0; k < VEC; ++k) {
            const int64_t e = g * VEC + k;
            int32_t a = aa[k], b = bb[k];
            bool act = e < m;
            if (act && ((uint32_t)a >= (uint64_t)n || (uint32_t)b >= (uint64_t)n)) {
                bad = true;
                act = false;
            }
            act = act && a != b;
            if (!act) a = b = 0;
            const uint64_t key = ((uint64_t)ww[k] << 32) | ((uint64_t)e << sh);
            const uint64_t key_b = key | (uint64_t)sh;
            bool act_a = act, act_b = act;
            if (act && (a == hot || b == hot)) {
                atomicMin(&s_hot, (unsigned long long)(a == hot ? key : key_b));
                act_a = a != hot;
                act_b = b != hot;
            }
            wave_min_update(best, a, key, act_a);
            wave_min_update(best, b, key_b, act_b);
        }
    }
    if (__ballot(bad) && lane_id() == 0) atomicOr(&ctrl->err, kErrRange);
    __syncthreads();
    if (threadIdx.x == 0 && hot >= 0 && s_hot != kKeyMax) atomic_min_key(&best[hot], s_hot);
}

// Round-0 minedge for graphs whose edges join nearby ids (the locality
// sample): each workgroup walks a contiguous run of tiles and keeps the minima
// of a window of kWinSlots consecutive vertex ids in LDS.  The window start
// only moves up (to just below each tile's first endpoint); the ids it leaves
// behind are written out with one atomic each, consecutive lanes on
// consecutive ids.  Endpoints outside the window take the global path, their
// reads issued together before the atomics.  Sorted-by-source edge lists (the
// usual layout of generated and distributed graphs) keep nearly every endpoint
// in the window; any other order is still correct, only slower.  Used when
// every workgroup that fits at once gets a tile (launch_minedge_r0).
constexpr int kWinThreads = 1024;
constexpr int kWinGroups = 2;                                   // 4-edge groups per lane per tile
constexpr int64_t kWinTile = (int64_t)kWinThreads * 4 * kWinGroups;   // 8192 edges
constexpr int64_t kWinSlots = 16384;                            // 128 KiB of minima
constexpr int64_t kWinSlack = kWinSlots / 8;                    // room below a tile's first id

// Writes the window's minima of ids [lo, hi) out (and clears them): one
// atomic per id that has a minimum, consecutive lanes on consecutive ids.  No
// read first: nearly every id is written out once.
__device__ __forceinline__ void win_flush(unsigned long long* s_min, uint64_t* best,
                                          int64_t lo, int64_t hi) {
    for (int64_t x = lo + threadIdx.x; x < hi; x += kWinThreads) {
        const int slot = (int)(x & (kWinSlots - 1));
        const uint64_t k = s_min[slot];
        if (k != kKeyMax) {
            s_min[slot] = kKeyMax;
            atomicMin((unsigned long long*)&best[x], (unsigned long long)k);
        }
    }
}

// The lane's 4-edge groups of tile t (positions past m read position m - 1,
// which the caller drops): 16-byte loads, the arrays 16-byte aligned.
__device__ __forceinline__ void win_load(const int32_t* __restrict__ u,
                                         const int32_t* __restrict__ v,
                                         const uint32_t* __restrict__ w, int64_t m, int64_t t,
                                         int32_t (&aa)[kWinGroups * 4],
                                         int32_t (&bb)[kWinGroups * 4],
                                         uint32_t (&ww)[kWinGroups * 4]) {
    const int64_t ng = m / 4;   // whole groups
#pragma unroll
    for (int j = 0; j < kWinGroups; ++j) {
        const int64_t g = t * (kWinTile / 4) + (int64_t)j * kWinThreads + threadIdx.x;
        if (g < ng) {
            const int4 a4 = reinterpret_cast<const int4*>(u)[g];
            const int4 b4 = reinterpret_cast<const int4*>(v)[g];
            const uint4 w4 = reinterpret_cast<const uint4*>(w)[g];
            aa[j * 4 + 0] = a4.x; aa[j * 4 + 1] = a4.y; aa[j * 4 + 2] = a4.z; aa[j * 4 + 3] = a4.w;
            bb[j * 4 + 0] = b4.x; bb[j * 4 + 1] = b4.y; bb[j * 4 + 2] = b4.z; bb[j * 4 + 3] = b4.w;
            ww[j * 4 + 0] = w4.x; ww[j * 4 + 1] = w4.y; ww[j * 4 + 2] = w4.z; ww[j * 4 + 3] = w4.w;
        } else {
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int64_t e = g * 4 + k < m ? g * 4 + k : m - 1;
                aa[j * 4 + k] = u[e];
                bb[j * 4 + k] = v[e];
                ww[j * 4 + k] = w[e];
            }
        }
    }
}

__global__ __launch_bounds__(kWinThreads) void k_minedge_win(
    const int32_t* __restrict__ u, const int32_t* __restrict__ v, const uint32_t* __restrict__ w,
    int64_t m, int64_t n, uint64_t* __restrict__ best, Ctrl* ctrl, int32_t hot,
    int64_t tiles_per_block, int sh) {
    __shared__ unsigned long long s_min[kWinSlots];
    __shared__ unsigned long long s_hot;
    __shared__ int64_t s_base;
    const int tid = threadIdx.x;
    for (int i = tid; i < kWinSlots; i += kWinThreads) s_min[i] = kKeyMax;
    if (tid == 0) s_hot = kKeyMax;
    const int64_t ntiles = (m + kWinTile - 1) / kWinTile;
    const int64_t t0 = (int64_t)blockIdx.x * tiles_per_block;
    const int64_t t1 = t0 + tiles_per_block < ntiles ? t0 + tiles_per_block : ntiles;
    int64_t base = -1;            // window [base, base + kWinSlots), the same in every thread
    bool bad = false;
    constexpr int kE = kWinGroups * 4;
    // the next tile is loaded while this one is decided
    int32_t na[kE], nb[kE];
    uint32_t nw[kE];
    if (t0 < t1) win_load(u, v, w, m, t0, na, nb, nw);
    for (int64_t t = t0; t < t1; ++t) {
        const int64_t e0 = t * kWinTile;
        int32_t aa[kE], bb[kE];
        uint32_t ww[kE];
#pragma unroll
        for (int i = 0; i < kE; ++i) { aa[i] = na[i]; bb[i] = nb[i]; ww[i] = nw[i]; }
        win_load(u, v, w, m, t + 1 < t1 ? t + 1 : t, na, nb, nw);
        if (tid == 0) {           // thread 0's first edge is the tile's first
            const uint32_t a0 = (uint32_t)aa[0], b0 = (uint32_t)bb[0];
            const int64_t f = (int64_t)(a0 < b0 ? a0 : b0);
            int64_t nbase = f < (int64_t)n ? f - kWinSlack : base;
            if (nbase < 0) nbase = 0;
            if (nbase < base) nbase = base;
            s_base = nbase;
        }
        __syncthreads();          // the last tile's LDS updates are done; s_base is set
        const int64_t nbase = s_base;
        if (base >= 0 && nbase > base)
            win_flush(s_min, best, base, nbase < base + kWinSlots ? nbase : base + kWinSlots);
        base = nbase;
        __syncthreads();          // the slots left behind are clear before they are reused
        uint64_t key[kE];
        bool ga[kE], gb[kE];      // endpoint takes the global path
#pragma unroll
        for (int i = 0; i < kE; ++i) {
            const int j = i / 4, k = i % 4;
            const int64_t e = (e0 / 4 + (int64_t)j * kWinThreads + tid) * 4 + k;
            int32_t a = aa[i], b = bb[i];
            bool act = e < m;
            if (act && ((uint32_t)a >= (uint64_t)n || (uint32_t)b >= (uint64_t)n)) {
                bad = true;
                act = false;
            }
            act = act && a != b;
            key[i] = ((uint64_t)ww[i] << 32) | ((uint64_t)e << sh);   // the a end's key
            const uint64_t key_b = key[i] | (uint64_t)sh;
            bool act_a = act, act_b = act;
            if (act && (a == hot || b == hot)) {
                atomicMin(&s_hot, (unsigned long long)(a == hot ? key[i] : key_b));
                act_a = a != hot;
                act_b = b != hot;
            }
            const uint64_t oa = (uint64_t)((int64_t)a - base), ob = (uint64_t)((int64_t)b - base);
            ga[i] = act_a && oa >= (uint64_t)kWinSlots;
            gb[i] = act_b && ob >= (uint64_t)kWinSlots;
            if (act_a && !ga[i]) {
                unsigned long long* p = &s_min[a & (kWinSlots - 1)];
                if (key[i] < *p) atomicMin(p, (unsigned long long)key[i]);
            }
            if (act_b && !gb[i]) {
                unsigned long long* p = &s_min[b & (kWinSlots - 1)];
                if (key_b < *p) atomicMin(p, (unsigned long long)key_b);
            }
            aa[i] = ga[i] ? a : 0;
            bb[i] = gb[i] ? b : 0;
        }
        // outside the window: every read first, then the atomics that still lower
        uint64_t ca[kE], cb[kE];
#pragma unroll
        for (int i = 0; i < kE; ++i) {
            ca[i] = ga[i] ? best[aa[i]] : 0;
            cb[i] = gb[i] ? best[bb[i]] : 0;
        }
#pragma unroll
        for (int i = 0; i < kE; ++i) {
            const uint64_t key_b = key[i] | (uint64_t)sh;
            wave_min_commit(best, aa[i], key[i], ga[i] && key[i] < ca[i]);
            wave_min_commit(best, bb[i], key_b, gb[i] && key_b < cb[i]);
        }
    }
    __syncthreads();
    if (base >= 0) win_flush(s_min, best, base, base + kWinSlots < n ? base + kWinSlots : n);
    if (__ballot(bad) && lane_id() == 0) atomicOr(&ctrl->err, kErrRange);
    if (tid == 0 && hot >= 0 && s_hot != kKeyMax) atomic_min_key(&best[hot], s_hot);
}

// ------------------------------------------------------------------ hook

// parent[x] = other endpoint of x's lightest edge.  Both vertices of a
// 2-cycle picked the same edge (strict order), recognised as best[other] ==
// best[x]; the smaller id is the root.  Every other live vertex owns exactly
// one MSF edge and marks it, so each MSF edge is counted once.  `cmap` maps
// the view's stored labels to this round's labels (null: identity).  SIDE:
// the keys are w << 32 | position << 1 | side (side 1: x is the edge's v
// end), so only the other end is read, and the other end's key for the same
// edge has the opposite side bit.  rootbits / livebits: bit x of word x / 64
// says whether x is a root that found an edge / found an edge at all (the
// root scan and the labelling read these instead of parent[] and best[]).
constexpr int kHookBlock = 1024;
template <int MODE, bool SIDE>
__global__ __launch_bounds__(kHookBlock) void k_hook(const uint64_t* __restrict__ best, int64_t nr,
                                                 View g, const int32_t* __restrict__ cmap,
                                                 int32_t* __restrict__ parent,
                                                 uint8_t* __restrict__ mask,
                                                 uint64_t* __restrict__ rootbits,
                                                 uint64_t* __restrict__ livebits, Ctrl* ctrl) {
    uint64_t wsum = 0, nfound = 0, nlive = 0;
    bool bad = false;
    // a wave's lanes take 64 consecutive vertices from a multiple of 64 (the
    // block size and the grid stride are multiples of 64), so lane 0 writes
    // the wave's root and live bits as one word each
    for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < nr;
         x += (int64_t)gridDim.x * blockDim.x) {
        bool live = false, root = false;
        do {
        const uint64_t b = best[x];
        if (b == kKeyMax) { parent[x] = (int32_t)x; break; }
        live = true;
        ++nlive;
        uint32_t pos;
        int32_t other;
        if constexpr (SIDE) {
            pos = (uint32_t)b >> 1;
            const bool at_v = (uint32_t)b & 1u;   // x is the edge's v end: u is the other
            if constexpr (MODE == kOrig) {
                // the caller's arrays are far larger than the caches: these
                // lines are read once, so non-temporal loads leave the caches
                // to best[]
                other = at_v ? __builtin_nontemporal_load(g.u + pos)
                             : __builtin_nontemporal_load(g.v + pos);
            } else if constexpr (MODE == kFull16) {
                const uint32_t p = g.p16[pos];
                other = (int32_t)(at_v ? (p & 0xffffu) : (p >> 16));
            } else {
                other = at_v ? g.u[pos] : g.v[pos];
            }
            if (cmap) other = cmap[other];
        } else {
            pos = (uint32_t)b;
            int32_t eu, ev;
            if constexpr (MODE == kOrig) {
                eu = __builtin_nontemporal_load(g.u + pos);
                ev = __builtin_nontemporal_load(g.v + pos);
            } else {
                load_ends<MODE>(g, pos, eu, ev);
            }
            if (cmap) { eu = cmap[eu]; ev = cmap[ev]; }
            if (eu != x && ev != x) bad = true;
            other = eu == (int32_t)x ? ev : eu;
        }
        if ((uint32_t)other >= (uint64_t)nr) { bad = true; parent[x] = (int32_t)x; break; }
        if (best[other] == (SIDE ? b ^ 1u : b) && (int32_t)x < other) {
            parent[x] = (int32_t)x;
            root = true;
        } else {
            parent[x] = other;
            mask[edge_id<MODE>(g, pos)] = 1;
            wsum += b >> 32;
            ++nfound;
        }
        } while (false);
        const uint64_t rb = __ballot(root), lb = __ballot(live);
        if (lane_id() == 0) {
            rootbits[x >> 6] = rb;
            livebits[x >> 6] = lb;
        }
    }
    // one set of counter atomics per workgroup (same-address atomics from
    // every wave would serialise)
    __shared__ uint64_t s_red[3][kHookBlock / kWave];
    __shared__ uint32_t s_bad;
    if (threadIdx.x == 0) s_bad = 0;
    wsum = wave_sum_u64(wsum);
    nfound = wave_sum_u64(nfound);
    nlive = wave_sum_u64(nlive);
    const int wave = threadIdx.x / kWave;
    __syncthreads();
    if (lane_id() == 0) {
        s_red[0][wave] = wsum;
        s_red[1][wave] = nfound;
        s_red[2][wave] = nlive;
    }
    if (__ballot(bad) && lane_id() == 0) s_bad = 1;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t a = 0, f = 0, l = 0;
        for (int i = 0; i < kHookBlock / kWave; ++i) {
            a += s_red[0][i];
            f += s_red[1][i];
            l += s_red[2][i];
        }
        if (f) {
            atomicAdd((unsigned long long*)&ctrl->total, (unsigned long long)a);
            atomicAdd((unsigned long long*)&ctrl->msf_edges, (unsigned long long)f);
            atomicAdd((unsigned long long*)&ctrl->found, (unsigned long long)f);
        }
        if (l) atomicAdd((unsigned long long*)&ctrl->live, (unsigned long long)l);
        if (s_bad) atomicOr(&ctrl->err, kErrInternal);
    }
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

// Dense ids for the roots that still have edges: stable scan over the hook's
// root bits; root x gets label[x] = its rank.
__global__ __launch_bounds__(kBlock) void k_scan_roots(
    const uint64_t* __restrict__ rootbits, int64_t nr,
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
        const int64_t x0 = wbase + k * kWave;          // a multiple of 64
        mk[k] = x0 < nr ? rootbits[x0 >> 6] : 0;
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
    const int32_t* __restrict__ parent, const uint64_t* __restrict__ livebits, int64_t nr,
    int32_t* __restrict__ label, uint64_t* __restrict__ best_next, const Ctrl* ctrl) {
    const int64_t nn = (int64_t)ctrl->n_next;
    for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < nr;
         x += (int64_t)gridDim.x * blockDim.x) {
        const int32_t p = parent[x];
        if (!((livebits[x >> 6] >> (x & 63)) & 1)) label[x] = -1;
        else if (p != (int32_t)x) label[x] = label[p];
        if (x < nn) best_next[x] = kKeyMax;
    }
}

// out[i] = label[cmap[i]] (-1 stays -1): the map from a view's stored labels
// to the next round's labels.
__global__ __launch_bounds__(kBlock) void k_compose(const int32_t* __restrict__ cmap, int64_t nc,
                                                    const int32_t* __restrict__ label,
                                                    int32_t* __restrict__ out) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nc;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t c = cmap[i];
        out[i] = c < 0 ? -1 : label[c];
    }
}

// Representative tracking for Filter-Borůvka (Sec. V: after a round every
// vertex records the component root it was contracted into; the chains are
// compressed by pointer doubling at the end).  orig_cur[x] is the input
// vertex that round vertex x stands for (null: identity).
__global__ __launch_bounds__(kBlock) void k_rep_update(
    const int32_t* __restrict__ parent, const uint64_t* __restrict__ livebits,
    const int32_t* __restrict__ label, int64_t nr, const int32_t* __restrict__ orig_cur,
    int32_t* __restrict__ orig_next, int32_t* __restrict__ rep) {
    for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < nr;
         x += (int64_t)gridDim.x * blockDim.x) {
        if (!((livebits[x >> 6] >> (x & 63)) & 1)) continue;   // no edge
        const int32_t p = parent[x];
        const int32_t ox = orig_cur ? orig_cur[x] : (int32_t)x;
        if (p != (int32_t)x) rep[ox] = orig_cur ? orig_cur[p] : p;
        else orig_next[label[x]] = ox;
    }
}

// ------------------------------------------------------------ streaming pass

// Relabel + next-round minedge over every position of the view, keeping the
// positions.  Each lane handles 4 consecutive positions per step (vector
// loads).  The map M (view labels -> next-round labels, nc entries) and the
// next round's best[] can be staged in LDS when small.  OUT selects what is
// written: nothing (the caller composes maps instead), int32 label pairs, or
// packed 16-bit label pairs.  Dead edges are written as (0, 0).
template <int IN>
__device__ __forceinline__ void load_group(const View& g, int64_t q, int64_t m, int32_t (&a)[4],
                                           int32_t (&b)[4], uint32_t (&w)[4]) {
    const int64_t e0 = q * 4;
    if (e0 + 3 < m) {
        if constexpr (IN == kFull16) {
            const uint4 p = reinterpret_cast<const uint4*>(g.p16)[q];
            a[0] = p.x & 0xffff; b[0] = p.x >> 16; a[1] = p.y & 0xffff; b[1] = p.y >> 16;
            a[2] = p.z & 0xffff; b[2] = p.z >> 16; a[3] = p.w & 0xffff; b[3] = p.w >> 16;
        } else {
            const int4 a4 = reinterpret_cast<const int4*>(g.u)[q];
            const int4 b4 = reinterpret_cast<const int4*>(g.v)[q];
            a[0] = a4.x; a[1] = a4.y; a[2] = a4.z; a[3] = a4.w;
            b[0] = b4.x; b[1] = b4.y; b[2] = b4.z; b[3] = b4.w;
        }
        const uint4 w4 = reinterpret_cast<const uint4*>(g.w)[q];
        w[0] = w4.x; w[1] = w4.y; w[2] = w4.z; w[3] = w4.w;
    } else {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            a[k] = b[k] = 0;
            w[k] = 0;
            if (e0 + k < m) {
                load_ends<IN>(g, e0 + k, a[k], b[k]);
                w[k] = g.w[e0 + k];
            }
        }
    }
}

// Relabel + next-round minedge over every position of the view, keeping the
// positions.  Each lane handles kPassGroups groups of 4 consecutive positions
// per step (16-byte vector loads, all issued before any is consumed).  The
// map M (view labels -> next-round labels, nc entries) and the next round's
// best[] can be staged in LDS when small; LDS_M stages the first km entries of
// M (all of it, or the prefix that fits: after a hot-first renumbering the
// most used labels come first).  OUT selects what is written:
// nothing (the caller composes maps instead), int32 label pairs, or packed
// 16-bit label pairs.  Dead edges are written as (0, 0).  PAIR (last pass
// before the tail): instead of the next minedge, keep the lightest edge of
// every vertex pair in a triangular table.
template <int IN, int OUT, bool LDS_M, bool LDS_B, bool PAIR>
__global__ __launch_bounds__(kPassBlock) void k_pass(View g, const int32_t* __restrict__ M,
                                                     int64_t nc, int32_t* __restrict__ ou,
                                                     int32_t* __restrict__ ov,
                                                     uint32_t* __restrict__ op16,
                                                     uint64_t* __restrict__ best_next, int64_t nn,
                                                     uint64_t* __restrict__ pairs, int64_t km,
                                                     const uint64_t* __restrict__ pair_hot,
                                                     Ctrl* ctrl, int sh) {
    extern __shared__ uint64_t lds[];
    uint64_t* s_best = lds;                                        // nn entries (LDS_B)
    int32_t* s_map = reinterpret_cast<int32_t*>(lds + (LDS_B ? nn : 0));  // km entries (LDS_M)
    if constexpr (LDS_B)
        for (int64_t i = threadIdx.x; i < nn; i += blockDim.x) s_best[i] = kKeyMax;
    if constexpr (LDS_M)
        for (int64_t i = threadIdx.x; i < km; i += blockDim.x) s_map[i] = M[i];
    // PAIR with pair_hot: the lightest edge of each pair among the first kp
    // labels (hot first after a renumbering) is kept in LDS, after the map,
    // and merged into the table once per workgroup.
    unsigned long long* s_pair =
        reinterpret_cast<unsigned long long*>(lds + (LDS_B ? nn : 0) + (LDS_M ? (km + 1) / 2 : 0));
    const int64_t kp = PAIR && pair_hot ? (*pair_hot < kPairHot ? (int64_t)*pair_hot : kPairHot) : 0;
    for (int64_t i = threadIdx.x; i < kp * (kp - 1) / 2; i += blockDim.x) s_pair[i] = kKeyMax;
    if constexpr (LDS_B || LDS_M || PAIR) __syncthreads();
    auto map = [&](int32_t a) -> int32_t {
        if constexpr (LDS_M) return a < km ? s_map[a] : M[a];
        else return M[a];
    };
    uint64_t* bst = LDS_B ? s_best : best_next;

    constexpr int G = kPassGroups;
    const int64_t m = g.len;
    const int64_t groups = (m + 3) / 4;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    // Skewed graphs leave a few huge components whose entries every lane
    // would update: the label most frequent among 64 sampled edges of this
    // workgroup's first positions (if it holds at least 1/8 of them) has its
    // minimum taken in LDS and merged once.  (PAIR has no per-vertex minimum.)
    __shared__ int32_t s_hot[kHot];
    __shared__ unsigned long long s_hotmin[kHot];
    if (!PAIR && threadIdx.x < kWave) {
        const int64_t p = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x * (blockDim.x / kWave)) * 4;
        int32_t lab = -1;
        if (p < m) {
            int32_t a0, b0;
            load_ends<IN>(g, p, a0, b0);
            if (a0 != b0) lab = map(a0);
        }
        hot_labels(lab, s_hot, s_hotmin);
    }
    __syncthreads();
    int32_t hot[kHot];
#pragma unroll
    for (int h = 0; h < kHot; ++h) hot[h] = PAIR ? -1 : s_hot[h];
    uint32_t kept = 0;
    // the loop bound is uniform per wave (wave_min_update needs whole waves)
    for (int64_t qw = blockIdx.x * (int64_t)blockDim.x + (threadIdx.x & ~(kWave - 1));
         qw < groups; qw += stride * G) {
        const int64_t q0 = qw + (threadIdx.x & (kWave - 1));
        int32_t a[G][4], b[G][4];
        uint32_t w[G][4];
#pragma unroll
        for (int j = 0; j < G; ++j) {
            const int64_t q = q0 + j * stride;
            if (q < groups) {
                load_group<IN>(g, q, m, a[j], b[j], w[j]);
            } else {
#pragma unroll
                for (int k = 0; k < 4; ++k) { a[j][k] = b[j][k] = 0; w[j][k] = 0; }
            }
        }
#pragma unroll
        for (int j = 0; j < G; ++j) {
            const int64_t q = q0 + j * stride;
            int32_t ra[4], rb[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                ra[k] = rb[k] = 0;
                bool act = false;
                uint64_t key = kKeyMax;
                if (q < groups && a[j][k] != b[j][k]) {   // equal stored labels stay a self-loop
                    const int32_t x = map(a[j][k]), y = map(b[j][k]);
                    if (x != y) {
                        ra[k] = x;
                        rb[k] = y;
                        ++kept;
                        act = true;
                        key = ((uint64_t)w[j][k] << 32) | ((uint64_t)(q * 4 + k) << (PAIR ? 0 : sh));
                        if constexpr (PAIR) {   // lightest edge per vertex pair, for the tail
                            const int64_t lo = x < y ? x : y, hi = x < y ? y : x;
                            const int64_t slot = hi * (hi - 1) / 2 + lo;
                            if (hi < kp) {
                                if (key < s_pair[slot]) atomicMin(&s_pair[slot], (unsigned long long)key);
                            } else {
                                atomic_min_key(&pairs[slot], key);
                            }
                        }
                    }
                }
                if constexpr (!PAIR) {   // the v end's key has the side bit (sh = 1)
                    const uint64_t key_b = key | (uint64_t)sh;
                    const bool hx = act && hot_min(hot, s_hotmin, ra[k], key);
                    const bool hy = act && hot_min(hot, s_hotmin, rb[k], key_b);
                    wave_min_update(bst, ra[k], key, act && !hx);
                    wave_min_update(bst, rb[k], key_b, act && !hy);
                }
            }
            if (q < groups) store_group<OUT>(q, m, ra, rb, ou, ov, op16);
        }
    }
    {   // one counter atomic per workgroup (same-address atomics queue)
        __shared__ uint64_t s_kept[kPassBlock / kWave];
        uint64_t tot;
        (void)block_excl_scan(kept, s_kept, &tot);
        if (threadIdx.x == 0 && tot)
            atomicAdd((unsigned long long*)&ctrl->m_next, (unsigned long long)tot);
    }
    if constexpr (!PAIR) {
        __syncthreads();
        if (threadIdx.x < kHot && hot[threadIdx.x] >= 0 && s_hotmin[threadIdx.x] != kKeyMax)
            atomic_min_key(&bst[hot[threadIdx.x]], s_hotmin[threadIdx.x]);
    } else {
        __syncthreads();
        for (int64_t i = threadIdx.x; i < kp * (kp - 1) / 2; i += blockDim.x)
            if (s_pair[i] != kKeyMax) atomic_min_key(&pairs[i], s_pair[i]);
    }
    if constexpr (LDS_B) {
        __syncthreads();
        for (int64_t i = threadIdx.x; i < nn; i += blockDim.x) {
            const uint64_t k = s_best[i];
            if (k != kKeyMax) atomic_min_key(&best_next[i], k);
        }
    }
}

// ----------------------------------------------------------- compaction pass

// Parallel-edge prefilter of one compaction tile (the hash-table prefilter of
// the paper's Sec. VI-B, held in LDS): every live relabelled edge enters its
// vertex pair into an open-addressing table and min-reduces its key (w << 32 |
// position; positions are in edge-id order) into the pair's entry; only the
// lightest edge of each pair in the tile survives.  A dropped edge has a
// lighter parallel edge, with which it closes a cycle on which it is the
// heaviest, so it is in no MSF (cycle property).  The table has twice as many
// slots as a tile has edges, so every probe sequence ends.
constexpr int kDedupSlots = 2 * kRelabelTile;
constexpr uint32_t kCompactGrid = 4096;   // workgroups of the compaction passes (tiles grid-stride)

template <uint32_t SLOTS = kDedupSlots>
__device__ __forceinline__ uint32_t pair_slot(uint64_t pair) {
    return (uint32_t)((pair * 0x9E3779B97F4A7C15ULL) >> 40) & (SLOTS - 1);
}

// Inserts `pair` (never kKeyMax) and min-reduces `key` into its entry; returns the slot.
// Plain reads first: a slot, once taken, keeps its pair, and an entry's minimum
// only falls, so a read showing the pair (or a minimum at most `key`) makes the
// atomic unnecessary; most edges of a tile meet a pair already entered.
template <uint32_t SLOTS = kDedupSlots>
__device__ __forceinline__ uint32_t dedup_insert(unsigned long long* s_pair,
                                                 unsigned long long* s_min, uint64_t pair,
                                                 uint64_t key) {
    uint32_t slot = pair_slot<SLOTS>(pair);
    for (uint32_t probe = 0; probe < SLOTS; ++probe) {
        unsigned long long cur = __hip_atomic_load(&s_pair[slot], __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_WORKGROUP);
        if (cur == kKeyMax)
            cur = atomicCAS(&s_pair[slot], (unsigned long long)kKeyMax, (unsigned long long)pair);
        if (cur == kKeyMax || cur == pair) break;
        slot = (slot + 1) & (SLOTS - 1);
    }
    if (key < __hip_atomic_load(&s_min[slot], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP))
        atomicMin(&s_min[slot], (unsigned long long)key);
    return slot;
}

// Exact parallel-edge removal: a global open-addressing table of vertex pairs
// (dslots entries, a power of two at least twice the edges) holds the
// lightest key of each pair over the whole view.
__device__ __forceinline__ uint64_t gpair_slot(uint64_t pair, int64_t dslots) {
    return ((pair * 0x9E3779B97F4A7C15ULL) >> 20) & (uint64_t)(dslots - 1);
}

template <int IN>
__global__ __launch_bounds__(kBlock) void k_dedup_insert(View g, const int32_t* __restrict__ M,
                                                         unsigned long long* dpair,
                                                         unsigned long long* dmin,
                                                         int64_t dslots) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < g.len;
         e += (int64_t)gridDim.x * blockDim.x) {
        int32_t a, b;
        load_ends<IN>(g, e, a, b);
        if (a == b) continue;
        a = M[a];
        b = M[b];
        if (a == b) continue;
        const uint64_t lo = (uint32_t)(a < b ? a : b), hi = (uint32_t)(a < b ? b : a);
        const uint64_t pair = (lo << 32) | hi;
        const uint64_t key = ((uint64_t)g.w[e] << 32) | (uint64_t)e;
        uint64_t slot = gpair_slot(pair, dslots);
        for (int64_t probe = 0; probe < dslots; ++probe) {
            const unsigned long long old = atomicCAS(&dpair[slot], (unsigned long long)kKeyMax,
                                                     (unsigned long long)pair);
            if (old == kKeyMax || old == pair) break;
            slot = (slot + 1) & (uint64_t)(dslots - 1);
        }
        if (key < dmin[slot]) atomicMin(&dmin[slot], (unsigned long long)key);
    }
}

// The lightest key of `pair` in the filled global table.
__device__ __forceinline__ uint64_t gpair_min(const uint64_t* dpair, const uint64_t* dmin,
                                              int64_t dslots, uint64_t pair) {
    uint64_t slot = gpair_slot(pair, dslots);
    for (int64_t probe = 0; probe < dslots; ++probe) {
        const uint64_t p = dpair[slot];
        if (p == pair) return dmin[slot];
        if (p == kKeyMax) break;              // not entered: cannot happen for a live edge
        slot = (slot + 1) & (uint64_t)(dslots - 1);
    }
    return kKeyMax;
}

// Compaction of the live edges after relabelling, in three steps with no
// waiting between tiles (reduce, scan, scatter):
//   k_compact_flags    relabel through M, drop self-loops and (DEDUP) every
//                      edge with a lighter parallel edge in its tile
//                      (kDedupLocal, the prefilter above) or in the whole view
//                      (kDedupExact, the global table); one keep bit per
//                      position and the kept count of every 2048-edge tile;
//   launch_scan_tiles  exclusive offsets of the tiles, the total to m_next;
//   k_compact_scatter  the kept edges, relabelled, stably at their offsets
//                      (position order stays edge-id order) and, FUSED, the
//                      next round's lightest-edge search on them with key
//                      w << 32 | new position << sh, the v end's | sh.
// Flag word i covers positions [64 i, 64 i + 64); tile t owns words
// [32 t, 32 t + 32), wave j of it words 32 t + 8 j + k.  `out` must not alias
// the view.
constexpr int kTileWords = kRelabelTile / kWave;

template <int IN, int DEDUP>
__global__ __launch_bounds__(kBlock) void k_compact_flags(View g, const int32_t* __restrict__ M,
                                                          uint64_t* __restrict__ flags,
                                                          uint64_t* __restrict__ cnt,
                                                          uint32_t ntiles, const uint64_t* dpair,
                                                          const uint64_t* dmin, int64_t dslots) {
    constexpr int kIt = kRelabelItems;
    constexpr int kTab = DEDUP == kDedupLocal ? kDedupSlots : 1;
    __shared__ uint32_t s_wave[kBlock / kWave];
    __shared__ unsigned long long s_pair[kTab];
    __shared__ unsigned long long s_min[kTab];
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int64_t mr = g.len;
    // A tile's ends and weights are loaded while the previous tile is being
    // decided (issued after its label gathers, so waiting for those does not
    // wait for them); past the end (also past the last tile) a lane reads
    // position mr - 1 and drops it.
    int32_t na[kIt], nb[kIt];
    uint32_t nw[kIt];
    auto load_tile = [&](uint32_t t) {
        const int64_t e0 = (int64_t)t * kRelabelTile + (int64_t)wave * (kWave * kIt) + lane;
#pragma unroll
        for (int k = 0; k < kIt; ++k) {
            const int64_t e = e0 + k * kWave < mr ? e0 + k * kWave : mr - 1;
            load_ends<IN>(g, e, na[k], nb[k]);
            nw[k] = 0;
            if constexpr (DEDUP != kDedupNone) nw[k] = g.w[e];
        }
    };
    if (blockIdx.x < ntiles) load_tile(blockIdx.x);
    for (uint32_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int64_t e0 = (int64_t)tile * kRelabelTile + (int64_t)wave * (kWave * kIt) + lane;
        if constexpr (DEDUP == kDedupLocal) {
            for (int i = threadIdx.x; i < kTab; i += kBlock) {
                s_pair[i] = kKeyMax;
                s_min[i] = kKeyMax;
            }
        }
        int32_t a[kIt], b[kIt];
        uint32_t wt[kIt];
        bool keep[kIt];
#pragma unroll
        for (int k = 0; k < kIt; ++k) {
            keep[k] = e0 + k * kWave < mr && na[k] != nb[k];
            a[k] = M[keep[k] ? na[k] : 0];
            b[k] = M[keep[k] ? nb[k] : 0];
            wt[k] = nw[k];
        }
        load_tile(tile + gridDim.x);     // unconditional: no branch for the waits to merge over
#pragma unroll
        for (int k = 0; k < kIt; ++k) keep[k] = keep[k] && a[k] != b[k];
        if constexpr (DEDUP == kDedupExact) {
#pragma unroll
            for (int k = 0; k < kIt; ++k) {
                if (keep[k]) {
                    const uint32_t lo = (uint32_t)(a[k] < b[k] ? a[k] : b[k]);
                    const uint32_t hi = (uint32_t)(a[k] < b[k] ? b[k] : a[k]);
                    const uint64_t key = ((uint64_t)wt[k] << 32) | (uint64_t)(e0 + k * kWave);
                    keep[k] = gpair_min(dpair, dmin, dslots, ((uint64_t)lo << 32) | hi) == key;
                }
            }
        }
        if constexpr (DEDUP == kDedupLocal) {
            __syncthreads();             // the table is clear
            uint32_t slot[kIt];
#pragma unroll
            for (int k = 0; k < kIt; ++k) {
                slot[k] = 0;
                if (keep[k]) {
                    const uint32_t lo = (uint32_t)(a[k] < b[k] ? a[k] : b[k]);
                    const uint32_t hi = (uint32_t)(a[k] < b[k] ? b[k] : a[k]);
                    const uint64_t key = ((uint64_t)wt[k] << 32) | (uint64_t)(e0 + k * kWave);
                    slot[k] = dedup_insert(s_pair, s_min, ((uint64_t)lo << 32) | hi, key);
                }
            }
            __syncthreads();
#pragma unroll
            for (int k = 0; k < kIt; ++k) {
                const uint64_t key = ((uint64_t)wt[k] << 32) | (uint64_t)(e0 + k * kWave);
                if (keep[k] && s_min[slot[k]] != key) keep[k] = false;
            }
        }
        uint32_t c = 0;
        const int64_t w0 = (int64_t)tile * kTileWords + wave * kIt;
#pragma unroll
        for (int k = 0; k < kIt; ++k) {
            const uint64_t mk = __ballot(keep[k]);
            if (lane == 0) flags[w0 + k] = mk;
            c += __popcll(mk);
        }
        if (lane == 0) s_wave[wave] = c;
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t sum = 0;
            for (int i = 0; i < kBlock / kWave; ++i) sum += s_wave[i];
            cnt[tile] = sum;
        }
        __syncthreads();                 // s_wave and the table are reused by the next tile
    }
}

// k_compact_flags with the per-tile parallel-edge table (kDedupLocal) for
// graphs with id locality: 16 waves decide four consecutive flag tiles per
// step (waves 4j..4j+3 tile j, each as in k_compact_flags) against one shared
// table of 8192 pairs in 128 KiB of LDS: twice the waves per CU of the
// 2048-edge version (which two 64 KiB tables limit to 8) and four times the
// edges over which a pair's lighter edge is found.  The table holds at most
// one entry per edge of the step, so probing always ends.
constexpr int kFwThreads = 1024;
constexpr int kFwTiles = kFwThreads / kBlock;                  // flag tiles per step
constexpr uint32_t kFwSlots = (uint32_t)kFwTiles * kRelabelTile;   // 8192

template <int IN>
__global__ __launch_bounds__(kFwThreads) void k_compact_flags_wide(
    View g, const int32_t* __restrict__ M, uint64_t* __restrict__ flags,
    uint64_t* __restrict__ cnt, uint32_t ntiles) {
    constexpr int kIt = kRelabelItems;
    __shared__ unsigned long long s_pair[kFwSlots];
    __shared__ unsigned long long s_min[kFwSlots];
    __shared__ uint32_t s_wave[kFwThreads / kWave];
    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid / kWave), lane = tid % kWave;
    const int sub = wave / (kBlock / kWave), wv = wave % (kBlock / kWave);
    const int64_t mr = g.len;
    const int64_t nsteps = ((int64_t)ntiles + kFwTiles - 1) / kFwTiles;
    // the next step's ends and weights load while this one is decided (past
    // the end a lane reads position mr - 1 and drops it)
    int32_t na[kIt], nb[kIt];
    uint32_t nw[kIt];
    auto load_step = [&](int64_t st) {
        const int64_t e0 = (st * kFwTiles + sub) * kRelabelTile + (int64_t)wv * (kWave * kIt) + lane;
#pragma unroll
        for (int k = 0; k < kIt; ++k) {
            const int64_t e = e0 + k * kWave < mr ? e0 + k * kWave : mr - 1;
            load_ends<IN>(g, e, na[k], nb[k]);
            nw[k] = g.w[e];
        }
    };
    if ((int64_t)blockIdx.x < nsteps) load_step(blockIdx.x);
    for (int64_t step = blockIdx.x; step < nsteps; step += gridDim.x) {
        const int64_t tile = step * kFwTiles + sub;
        const int64_t e0 = tile * kRelabelTile + (int64_t)wv * (kWave * kIt) + lane;
        for (uint32_t i = tid; i < kFwSlots; i += kFwThreads) {
            s_pair[i] = kKeyMax;
            s_min[i] = kKeyMax;
        }
        int32_t a[kIt], b[kIt];
        uint32_t wt[kIt];
        bool keep[kIt];
#pragma unroll
        for (int k = 0; k < kIt; ++k) {
            keep[k] = e0 + k * kWave < mr && na[k] != nb[k];
            a[k] = M[keep[k] ? na[k] : 0];
            b[k] = M[keep[k] ? nb[k] : 0];
            wt[k] = nw[k];
        }
        load_step(step + gridDim.x);     // unconditional: no branch for the waits to merge over
#pragma unroll
        for (int k = 0; k < kIt; ++k) keep[k] = keep[k] && a[k] != b[k];
        __syncthreads();                 // the table is clear
        uint32_t slot[kIt];
#pragma unroll
        for (int k = 0; k < kIt; ++k) {
            slot[k] = 0;
            if (keep[k]) {
                const uint32_t lo = (uint32_t)(a[k] < b[k] ? a[k] : b[k]);
                const uint32_t hi = (uint32_t)(a[k] < b[k] ? b[k] : a[k]);
                const uint64_t key = ((uint64_t)wt[k] << 32) | (uint64_t)(e0 + k * kWave);
                slot[k] = dedup_insert<kFwSlots>(s_pair, s_min, ((uint64_t)lo << 32) | hi, key);
            }
        }
        __syncthreads();
        uint32_t c = 0;
        const int64_t w0 = tile * kTileWords + wv * kIt;
#pragma unroll
        for (int k = 0; k < kIt; ++k) {
            const uint64_t key = ((uint64_t)wt[k] << 32) | (uint64_t)(e0 + k * kWave);
            const bool kp = keep[k] && s_min[slot[k]] == key;
            const uint64_t mk = __ballot(kp);
            if (lane == 0 && tile < (int64_t)ntiles) flags[w0 + k] = mk;
            c += __popcll(mk);
        }
        if (lane == 0) s_wave[wave] = c;
        __syncthreads();
        if (tid < kFwTiles && step * kFwTiles + tid < (int64_t)ntiles) {
            uint32_t sum = 0;
            for (int i = 0; i < kBlock / kWave; ++i) sum += s_wave[tid * (kBlock / kWave) + i];
            cnt[step * kFwTiles + tid] = sum;
        }
        __syncthreads();                 // s_wave and the table are reused by the next step
    }
}

template <int IN, bool FUSED>
__global__ __launch_bounds__(kBlock) void k_compact_scatter(View g, const int32_t* __restrict__ M,
                                                            const uint64_t* __restrict__ flags,
                                                            const uint64_t* __restrict__ off,
                                                            EdgeSoA out,
                                                            uint64_t* __restrict__ best_next,
                                                            uint32_t ntiles, int sh) {
    constexpr int kIt = kRelabelItems;
    __shared__ uint32_t s_wave[kBlock / kWave];
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    for (uint32_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int64_t w0 = (int64_t)tile * kTileWords + wave * kIt;
        const int64_t e0 = (int64_t)tile * kRelabelTile + (int64_t)wave * (kWave * kIt) + lane;
        uint64_t mk[kIt];
        uint32_t c = 0;
#pragma unroll
        for (int k = 0; k < kIt; ++k) {
            mk[k] = flags[w0 + k];
            c += __popcll(mk[k]);
        }
        if (lane == 0) s_wave[wave] = c;
        __syncthreads();
        uint32_t woff = 0;
#pragma unroll
        for (int i = 0; i < kBlock / kWave; ++i)
            if (i < wave) woff += s_wave[i];
        // all loads, then the label gathers, then the stores: the chains of
        // the scattered kept edges overlap
        int32_t a[kIt], b[kIt];
        uint32_t wt[kIt], id[kIt];
#pragma unroll
        for (int k = 0; k < kIt; ++k) {
            a[k] = b[k] = 0;
            wt[k] = id[k] = 0;
            if ((mk[k] >> lane) & 1) {
                const int64_t e = e0 + k * kWave;
                load_ends<IN>(g, e, a[k], b[k]);
                wt[k] = g.w[e];
                id[k] = edge_id<IN>(g, e);
            }
        }
#pragma unroll
        for (int k = 0; k < kIt; ++k) {
            if ((mk[k] >> lane) & 1) {
                a[k] = M[a[k]];
                b[k] = M[b[k]];
            }
        }
        uint64_t o = off[tile] + woff;
#pragma unroll
        for (int k = 0; k < kIt; ++k) {
            const bool kept = (mk[k] >> lane) & 1;
            const uint64_t d = o + lanes_below(mk[k]);
            if (kept) {
                out.u[d] = a[k];
                out.v[d] = b[k];
                out.w[d] = wt[k];
                out.id[d] = id[k];
            }
            if constexpr (FUSED) {   // the v end's key has the side bit (sh = 1)
                const uint64_t key = ((uint64_t)wt[k] << 32) | (d << sh);
                wave_min_update(best_next, a[k], key, kept);
                wave_min_update(best_next, b[k], key | (uint64_t)sh, kept);
            }
            o += __popcll(mk[k]);
        }
        __syncthreads();                 // s_wave is reused by the next tile
    }
}

// k_compact_scatter for graphs with id locality: the kept edges' new labels
// stay close together along the positions, so the next round's minima are
// taken in a sliding LDS window of labels (as in k_minedge_win) instead of one
// global update per endpoint.  A workgroup of 16 waves handles four
// consecutive flag tiles per step (waves 4j..4j+3 tile j, each as in
// k_compact_scatter) over a contiguous run of steps.  Same output.
constexpr int kSwThreads = 1024;
constexpr int kSwTiles = kSwThreads / kBlock;                 // flag tiles per step
constexpr int64_t kSwSlots = 8192;                            // 64 KiB of minima
constexpr int64_t kSwSlack = kSwSlots / 8;

// One step's flag words and (every position, past the end position
// len - 1) ends, weights and ids of the calling lane, for k_compact_scatter_win.
template <int IN>
__device__ __forceinline__ void sw_load(const View& g, const uint64_t* __restrict__ flags,
                                        uint32_t ntiles, int64_t step, int sub, int wv, int lane,
                                        uint64_t (&mk)[kRelabelItems],
                                        int32_t (&a)[kRelabelItems], int32_t (&b)[kRelabelItems],
                                        uint32_t (&wt)[kRelabelItems],
                                        uint32_t (&id)[kRelabelItems]) {
    constexpr int kIt = kRelabelItems;
    const int64_t tile = step * kSwTiles + sub;
    const bool live = tile < (int64_t)ntiles;
    const int64_t w0 = tile * kTileWords + wv * kIt;
    const int64_t e0 = tile * kRelabelTile + (int64_t)wv * (kWave * kIt) + lane;
#pragma unroll
    for (int k = 0; k < kIt; ++k) {
        mk[k] = live ? flags[w0 + k] : 0;
        const int64_t e = e0 + k * kWave < g.len ? e0 + k * kWave : g.len - 1;
        load_ends<IN>(g, e, a[k], b[k]);
        wt[k] = g.w[e];
        id[k] = edge_id<IN>(g, e);
    }
}

template <int IN>
__global__ __launch_bounds__(kSwThreads) void k_compact_scatter_win(
    View g, const int32_t* __restrict__ M, const uint64_t* __restrict__ flags,
    const uint64_t* __restrict__ off, EdgeSoA out, uint64_t* __restrict__ best_next,
    uint32_t ntiles, int64_t nn, int64_t steps_per_block, int sh) {
    constexpr int kIt = kRelabelItems;
    __shared__ unsigned long long s_min[kSwSlots];
    __shared__ uint32_t s_wave[kSwThreads / kWave];
    __shared__ int64_t s_base;
    const int tid = threadIdx.x;
    // the wave index as a wave-uniform value: the flag words become scalar loads
    const int wave = __builtin_amdgcn_readfirstlane(tid / kWave), lane = tid % kWave;
    const int sub = wave / (kBlock / kWave), wv = wave % (kBlock / kWave);
    for (int i = tid; i < kSwSlots; i += kSwThreads) s_min[i] = kKeyMax;
    const int64_t nsteps = ((int64_t)ntiles + kSwTiles - 1) / kSwTiles;
    const int64_t s0 = (int64_t)blockIdx.x * steps_per_block;
    const int64_t s1 = s0 + steps_per_block < nsteps ? s0 + steps_per_block : nsteps;
    int64_t base = -1;            // label window [base, base + kSwSlots), uniform
    // the next step is loaded while this one is decided (issued after this
    // step's label gathers, so waiting for those does not wait for it)
    uint64_t nmk[kIt];
    int32_t na[kIt], nb[kIt];
    uint32_t nw[kIt], nid[kIt];
    if (s0 < s1) sw_load<IN>(g, flags, ntiles, s0, sub, wv, lane, nmk, na, nb, nw, nid);
    for (int64_t step = s0; step < s1; ++step) {
        const int64_t tile = step * kSwTiles + sub;
        uint64_t mk[kIt];
        int32_t a[kIt], b[kIt];
        uint32_t wt[kIt], id[kIt];
        uint32_t c = 0;
#pragma unroll
        for (int k = 0; k < kIt; ++k) {
            mk[k] = nmk[k];
            wt[k] = nw[k];
            id[k] = nid[k];
            c += __popcll(mk[k]);
            // kept ends are relabelled; the others read M[0] (one request per
            // wave), except thread 0's first, whose label places the window
            const bool kept = (mk[k] >> lane) & 1;
            a[k] = M[kept || (k == 0 && tid == 0) ? na[k] : 0];
            b[k] = M[kept ? nb[k] : 0];
        }
        sw_load<IN>(g, flags, ntiles, step + 1 < s1 ? step + 1 : step, sub, wv, lane, nmk, na, nb,
                    nw, nid);
        if (lane == 0) s_wave[wave] = c;
        if (tid == 0) {           // below the label of the step's first position
            int64_t nbase = a[0] >= 0 && a[0] < nn ? (int64_t)a[0] - kSwSlack : base;
            if (nbase < 0) nbase = 0;
            if (nbase < base) nbase = base;
            s_base = nbase;
        }
        __syncthreads();          // the last step's LDS updates are done; counts and s_base set
        const int64_t nbase = s_base;
        if (base >= 0 && nbase > base) {
            const int64_t hi = nbase < base + kSwSlots ? nbase : base + kSwSlots;
            for (int64_t x = base + tid; x < hi; x += kSwThreads) {
                const int slot = (int)(x & (kSwSlots - 1));
                const uint64_t k = s_min[slot];
                if (k != kKeyMax) {
                    s_min[slot] = kKeyMax;
                    atomicMin((unsigned long long*)&best_next[x], (unsigned long long)k);
                }
            }
        }
        base = nbase;
        uint32_t woff = 0;
#pragma unroll
        for (int i = 0; i < kBlock / kWave; ++i)
            if (i < wv) woff += s_wave[sub * (kBlock / kWave) + i];
        __syncthreads();          // the slots left behind are clear
        uint64_t o = (tile < (int64_t)ntiles ? off[tile] : 0) + woff;
        uint64_t key[kIt];
        bool ga[kIt], gb[kIt];
#pragma unroll
        for (int k = 0; k < kIt; ++k) {
            const bool kept = (mk[k] >> lane) & 1;
            const uint64_t d = o + lanes_below(mk[k]);
            key[k] = ((uint64_t)wt[k] << 32) | (d << sh);   // the a end's; the b end's adds sh
            ga[k] = gb[k] = false;
            if (kept) {
                out.u[d] = a[k];
                out.v[d] = b[k];
                out.w[d] = wt[k];
                out.id[d] = id[k];
                const uint64_t oa = (uint64_t)((int64_t)a[k] - base);
                const uint64_t ob = (uint64_t)((int64_t)b[k] - base);
                ga[k] = oa >= (uint64_t)kSwSlots;
                gb[k] = ob >= (uint64_t)kSwSlots;
                if (!ga[k]) {
                    unsigned long long* p = &s_min[a[k] & (kSwSlots - 1)];
                    if (key[k] < *p) atomicMin(p, (unsigned long long)key[k]);
                }
                if (!gb[k]) {
                    const uint64_t kb = key[k] | (uint64_t)sh;
                    unsigned long long* p = &s_min[b[k] & (kSwSlots - 1)];
                    if (kb < *p) atomicMin(p, (unsigned long long)kb);
                }
            }
            if (!ga[k]) a[k] = 0;
            if (!gb[k]) b[k] = 0;
            o += __popcll(mk[k]);
        }
        // outside the window: every read first, then the atomics that still lower
        uint64_t ca[kIt], cb[kIt];
#pragma unroll
        for (int k = 0; k < kIt; ++k) {
            ca[k] = ga[k] ? best_next[a[k]] : 0;
            cb[k] = gb[k] ? best_next[b[k]] : 0;
        }
#pragma unroll
        for (int k = 0; k < kIt; ++k) {
            const uint64_t kb = key[k] | (uint64_t)sh;
            wave_min_commit(best_next, a[k], key[k], ga[k] && key[k] < ca[k]);
            wave_min_commit(best_next, b[k], kb, gb[k] && kb < cb[k]);
        }
    }
    __syncthreads();
    if (base >= 0) {
        const int64_t hi = base + kSwSlots < nn ? base + kSwSlots : nn;
        for (int64_t x = base + tid; x < hi; x += kSwThreads) {
            const uint64_t k = s_min[x & (kSwSlots - 1)];
            if (k != kKeyMax) atomicMin((unsigned long long*)&best_next[x], (unsigned long long)k);
        }
    }
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
// Compute units of the current device (cached per device).
static int64_t device_cus() {
    static std::atomic<int> cache[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    int c = cache[dev].load(std::memory_order_relaxed);
    if (c <= 0) {
        if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            c <= 0)
            c = 256;
        cache[dev].store(c, std::memory_order_relaxed);
    }
    return c;
}

// Workgroups of `kernel` that fit on the device at once.
template <typename K>
static int64_t resident_blocks(K kernel, int threads) {
    int per = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, threads, 0) != hipSuccess ||
        per < 1)
        per = 1;
    return per * device_cus();
}

void launch_minedge_r0(const int32_t* u, const int32_t* v, const uint32_t* w, int64_t m,
                       int64_t n, uint64_t* best, Ctrl* ctrl, int32_t hot, bool local,
                       bool side_keys, hipStream_t s) {
    if (m <= 0) return;
    if (hot >= n) hot = -1;
    const int sh = side_keys && m <= kSideKeyMaxEdges ? 1 : 0;
    const bool aligned = (((uintptr_t)u | (uintptr_t)v | (uintptr_t)w) & 15) == 0;
    // the window needs a tile for every workgroup that fits at once (one per
    // CU: the window takes 128 KiB of LDS); smaller graphs would leave most of
    // the chip idle, and the grid-stride kernel below spreads them wider
    const int64_t ntiles = (m + kWinTile - 1) / kWinTile;
    const int64_t cap = local && aligned ? resident_blocks(k_minedge_win, kWinThreads) : 0;
    if (local && aligned && ntiles >= cap) {
        const int64_t per = (ntiles + cap - 1) / cap;   // a contiguous run of tiles each
        hipLaunchKernelGGL(k_minedge_win, dim3((unsigned)((ntiles + per - 1) / per)),
                           dim3(kWinThreads), 0, s, u, v, w, m, n, best, ctrl, hot, per, sh);
        return;
    }
    if (aligned)
        hipLaunchKernelGGL(k_minedge_r0<4>, dim3(grid_for((m + 3) / 4)), dim3(kBlock), 0, s, u,
                           v, w, m, n, best, ctrl, hot, sh);
    else
        hipLaunchKernelGGL(k_minedge_r0<1>, dim3(grid_for(m)), dim3(kBlock), 0, s, u, v, w, m,
                           n, best, ctrl, hot, sh);
}
void launch_hook(int mode, const uint64_t* best, int64_t nr, const View& g, const int32_t* cmap,
                 int32_t* parent, uint8_t* mask, uint64_t* rootbits, uint64_t* livebits,
                 Ctrl* ctrl, bool side_keys, hipStream_t s) {
    int64_t hb = (nr + kHookBlock - 1) / kHookBlock;
    hb = hb < 1 ? 1 : (hb > 256 ? 256 : hb);
    const dim3 gr((unsigned)hb), bl(kHookBlock);
    if (side_keys) {
        switch (mode) {
            case kOrig: hipLaunchKernelGGL((k_hook<kOrig, true>), gr, bl, 0, s, best, nr, g, cmap, parent, mask, rootbits, livebits, ctrl); break;
            case kFull32: hipLaunchKernelGGL((k_hook<kFull32, true>), gr, bl, 0, s, best, nr, g, cmap, parent, mask, rootbits, livebits, ctrl); break;
            case kFull16: hipLaunchKernelGGL((k_hook<kFull16, true>), gr, bl, 0, s, best, nr, g, cmap, parent, mask, rootbits, livebits, ctrl); break;
            default: hipLaunchKernelGGL((k_hook<kCompact, true>), gr, bl, 0, s, best, nr, g, cmap, parent, mask, rootbits, livebits, ctrl); break;
        }
        return;
    }
    switch (mode) {
        case kOrig: hipLaunchKernelGGL((k_hook<kOrig, false>), gr, bl, 0, s, best, nr, g, cmap, parent, mask, rootbits, livebits, ctrl); break;
        case kFull32: hipLaunchKernelGGL((k_hook<kFull32, false>), gr, bl, 0, s, best, nr, g, cmap, parent, mask, rootbits, livebits, ctrl); break;
        case kFull16: hipLaunchKernelGGL((k_hook<kFull16, false>), gr, bl, 0, s, best, nr, g, cmap, parent, mask, rootbits, livebits, ctrl); break;
        default: hipLaunchKernelGGL((k_hook<kCompact, false>), gr, bl, 0, s, best, nr, g, cmap, parent, mask, rootbits, livebits, ctrl); break;
    }
}
void launch_jump(int32_t* parent, int64_t nr, int iters, Ctrl* ctrl, hipStream_t s) {
    hipLaunchKernelGGL(k_jump, dim3(grid_for(nr)), dim3(kBlock), 0, s, parent, nr, iters, ctrl);
}
void launch_scan_roots(const uint64_t* rootbits, int64_t nr, int32_t* label,
                       uint64_t* status, Ctrl* ctrl, hipStream_t s) {
    const uint32_t nt = (uint32_t)((nr + kTile - 1) / kTile);
    hipLaunchKernelGGL(k_scan_roots, dim3(nt), dim3(kBlock), 0, s, rootbits, nr, label,
                       status, ctrl, nt);
}
void launch_label(const int32_t* parent, const uint64_t* livebits, int64_t nr, int32_t* label,
                  uint64_t* best_next, const Ctrl* ctrl, hipStream_t s) {
    hipLaunchKernelGGL(k_label, dim3(grid_for(nr)), dim3(kBlock), 0, s, parent, livebits, nr, label,
                       best_next, ctrl);
}
void launch_compose(const int32_t* cmap, int64_t nc, const int32_t* label, int32_t* out,
                    hipStream_t s) {
    if (nc > 0)
        hipLaunchKernelGGL(k_compose, dim3(grid_for(nc)), dim3(kBlock), 0, s, cmap, nc, label, out);
}

// Hot-first renumbering before the tail (nn <= kTailMax labels): one
// workgroup samples kPreTailSample edge ends of the view (positions from the
// SplitMix64 output function of the sample index), takes each end's label
// lab[c] (c = the end's current vertex, through cmap when maps are composed),
// counts the samples per label in LDS, sorts the labels by count (most
// sampled first, ties by label), and writes the permutation in that order
// (perm[nn]) and the number of labels sampled at least once (*hot).
constexpr int kPreTailSample = 8192;
static_assert(kTailThreads >= kTailMax, "one thread per label");

template <int MODE>
__global__ __launch_bounds__(kTailThreads) void k_hot_first_small(
    View g, const int32_t* __restrict__ cmap, const int32_t* __restrict__ lab, int64_t nr,
    int64_t nn, int32_t* __restrict__ perm, uint64_t* __restrict__ hot) {
    __shared__ uint32_t s_cnt[kTailMax];
    __shared__ uint64_t s_key[kTailMax];
    __shared__ uint64_t s_w[kTailThreads / kWave];
    const int tid = threadIdx.x;
    if (tid < kTailMax) s_cnt[tid] = 0;
    __syncthreads();
    for (int i = tid; i < kPreTailSample; i += blockDim.x) {
        uint64_t z = (uint64_t)i * 0x9E3779B97F4A7C15ull + 0x13198A2E03707344ull;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z ^= z >> 31;
        const int64_t e = (int64_t)__umul64hi(z, (uint64_t)g.len);
        int32_t a, b;
        load_ends<MODE>(g, e, a, b);
        if (a != b) {
            const int32_t ca = cmap ? cmap[a] : a, cb = cmap ? cmap[b] : b;
            if (ca >= 0 && cb >= 0 && ca < nr && cb < nr) {
                const int32_t la = lab[ca], lb = lab[cb];
                const int32_t l = (i & 1) ? lb : la;
                if (la != lb && l >= 0 && l < nn) atomicAdd(&s_cnt[l], 1u);
            }
        }
    }
    __syncthreads();
    // sort key: fewer samples sort later, then the label (ascending sort)
    if (tid < kTailMax)
        s_key[tid] = tid < nn ? ((uint64_t)(0xffffffffu - s_cnt[tid]) << 32) | (uint64_t)tid
                              : ~0ull;
    const uint32_t f = tid < nn && s_cnt[tid] > 0 ? 1u : 0u;
    __syncthreads();
    for (int k = 2; k <= kTailMax; k <<= 1) {          // bitonic sort, ascending
        for (int jj = k >> 1; jj > 0; jj >>= 1) {
            if (tid < kTailMax) {
                const int p = tid ^ jj;
                if (p > tid) {
                    const uint64_t x = s_key[tid], y = s_key[p];
                    if (((tid & k) == 0) == (x > y)) { s_key[tid] = y; s_key[p] = x; }
                }
            }
            __syncthreads();
        }
    }
    uint64_t H;
    (void)block_excl_scan((uint64_t)f, s_w, &H);
    if (tid < nn) perm[(uint32_t)s_key[tid]] = tid;
    if (tid == 0) *hot = H;
}

__global__ __launch_bounds__(kBlock) void k_apply_perm(int32_t* __restrict__ lab, int64_t nr,
                                                       const int32_t* __restrict__ perm,
                                                       int64_t nn) {
    for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < nr;
         x += (int64_t)gridDim.x * blockDim.x) {
        const int32_t l = lab[x];
        if (l >= 0 && l < nn) lab[x] = perm[l];
    }
}

void launch_hot_first_small(int mode, const View& g, const int32_t* cmap, int32_t* lab, int64_t nr,
                            int64_t nn, int32_t* perm, uint64_t* hot, hipStream_t s) {
    if (g.len <= 0 || nn > kTailMax) return;
    const dim3 one(1), tb(kTailThreads);
    switch (mode) {
        case kOrig: hipLaunchKernelGGL(k_hot_first_small<kOrig>, one, tb, 0, s, g, cmap, lab, nr, nn, perm, hot); break;
        case kFull32: hipLaunchKernelGGL(k_hot_first_small<kFull32>, one, tb, 0, s, g, cmap, lab, nr, nn, perm, hot); break;
        case kFull16: hipLaunchKernelGGL(k_hot_first_small<kFull16>, one, tb, 0, s, g, cmap, lab, nr, nn, perm, hot); break;
        default: hipLaunchKernelGGL(k_hot_first_small<kCompact>, one, tb, 0, s, g, cmap, lab, nr, nn, perm, hot); break;
    }
    hipLaunchKernelGGL(k_apply_perm, dim3(grid_for(nr)), dim3(kBlock), 0, s, lab, nr, perm, nn);
}

void launch_rep_update(const int32_t* parent, const uint64_t* livebits, const int32_t* label,
                       int64_t nr, const int32_t* orig_cur, int32_t* orig_next, int32_t* rep,
                       hipStream_t s) {
    hipLaunchKernelGGL(k_rep_update, dim3(grid_for(nr)), dim3(kBlock), 0, s, parent, livebits, label,
                       nr, orig_cur, orig_next, rep);
}

// LDS budget of one pass workgroup: one per CU (its 16 waves are all the
// registers allow), so one copy of the minima and the map per CU.
constexpr int64_t kPassLds = 156 * 1024;
// Smallest map prefix worth staging when the whole map does not fit.
constexpr int64_t kMapPrefixMin = 1024;

// Raises the dynamic-LDS limit of one pass instantiation once (needed above
// 64 KiB); returns false when the runtime refuses.
template <int IN, int OUT, bool LM, bool LB, bool PAIR>
static bool allow_lds(size_t bytes) {
    if (bytes <= 64 * 1024) return true;
    static bool tried = false, ok = false;
    if (!tried) {
        tried = true;
        ok = hipFuncSetAttribute((const void*)k_pass<IN, OUT, LM, LB, PAIR>,
                                 hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)kPassLds) == hipSuccess;
        if (!ok) (void)hipGetLastError();
    }
    return ok;
}

template <int IN, int OUT, bool PAIR>
static void pass_dispatch(const View& g, const int32_t* M, int64_t nc, int32_t* ou, int32_t* ov,
                          uint32_t* op16, uint64_t* best_next, int64_t nn, uint64_t* pairs,
                          const uint64_t* pair_hot, Ctrl* ctrl, int sh, hipStream_t s) {
    const bool lds_on = true;
    bool ldsb = false;
    int64_t km = 0;
    size_t lds = 0;
    int64_t ptab = 0;
    for (int64_t budget : {kPassLds, (int64_t)64 * 1024}) {   // the second if the runtime refuses
        const int64_t want_ptab = kPairHot * (kPairHot - 1) / 2 * 8;
        ptab = PAIR && pair_hot && lds_on && want_ptab + 8 <= budget ? want_ptab : 0;
        ldsb = lds_on && !PAIR && nn * 8 <= budget;
        const int64_t left = budget - (ldsb ? nn * 8 : 0) - ptab - 8;
        km = !lds_on ? 0 : nc * 4 <= left ? nc : (left / 4 >= kMapPrefixMin ? left / 4 : 0);
        lds = (ldsb ? nn * 8 : 0) + (km + 1) / 2 * 8 + ptab;
        bool ok = true;
        if (ldsb && km) ok = allow_lds<IN, OUT, true, true, PAIR>(lds);
        else if (ldsb) ok = allow_lds<IN, OUT, false, true, PAIR>(lds);
        else if (km) ok = allow_lds<IN, OUT, true, false, PAIR>(lds);
        else ok = allow_lds<IN, OUT, false, false, PAIR>(lds);
        if (ok) break;
    }
    if (!ptab) pair_hot = nullptr;   // the kernel keeps LDS pairs only when given pair_hot
    const int64_t groups = (g.len + 3) / 4;
    int64_t want = (groups + (int64_t)kPassBlock * kPassGroups - 1) / ((int64_t)kPassBlock * kPassGroups);
    const int64_t cap = lds ? 256 : 512;   // LDS variants: one workgroup per CU
    const unsigned grid = (unsigned)(want < 1 ? 1 : (want > cap ? cap : want));
    const dim3 bl(kPassBlock);
    if (ldsb && km)
        hipLaunchKernelGGL((k_pass<IN, OUT, true, true, PAIR>), dim3(grid), bl, lds, s, g, M, nc, ou, ov, op16, best_next, nn, pairs, km, pair_hot, ctrl, sh);
    else if (ldsb)
        hipLaunchKernelGGL((k_pass<IN, OUT, false, true, PAIR>), dim3(grid), bl, lds, s, g, M, nc, ou, ov, op16, best_next, nn, pairs, km, pair_hot, ctrl, sh);
    else if (km)
        hipLaunchKernelGGL((k_pass<IN, OUT, true, false, PAIR>), dim3(grid), bl, lds, s, g, M, nc, ou, ov, op16, best_next, nn, pairs, km, pair_hot, ctrl, sh);
    else
        hipLaunchKernelGGL((k_pass<IN, OUT, false, false, PAIR>), dim3(grid), bl, lds, s, g, M, nc, ou, ov, op16, best_next, nn, pairs, km, pair_hot, ctrl, sh);
}

// Streaming pass; returns false for a layout/output pair it does not support.
// pairs != null: last pass before the tail (output kOutNone only).
bool launch_pass(int in_mode, int out, const View& g, const int32_t* M, int64_t nc, int32_t* ou,
                 int32_t* ov, uint32_t* op16, uint64_t* best_next, int64_t nn, uint64_t* pairs,
                 const uint64_t* pair_hot, Ctrl* ctrl, bool side_keys, hipStream_t s) {
    if (g.len <= 0) return true;
    const int sh = side_keys ? 1 : 0;
    if (pairs) {
        if (out != kOutNone) return false;
        switch (in_mode) {
            case kOrig: pass_dispatch<kOrig, kOutNone, true>(g, M, nc, ou, ov, op16, best_next, nn, pairs, pair_hot, ctrl, sh, s); return true;
            case kFull32: pass_dispatch<kFull32, kOutNone, true>(g, M, nc, ou, ov, op16, best_next, nn, pairs, pair_hot, ctrl, sh, s); return true;
            case kFull16: pass_dispatch<kFull16, kOutNone, true>(g, M, nc, ou, ov, op16, best_next, nn, pairs, pair_hot, ctrl, sh, s); return true;
            default: pass_dispatch<kCompact, kOutNone, true>(g, M, nc, ou, ov, op16, best_next, nn, pairs, pair_hot, ctrl, sh, s); return true;
        }
    }
    switch (in_mode * 3 + out) {
        case kOrig * 3 + kOut32: pass_dispatch<kOrig, kOut32, false>(g, M, nc, ou, ov, op16, best_next, nn, nullptr, nullptr, ctrl, sh, s); return true;
        case kOrig * 3 + kOut16: pass_dispatch<kOrig, kOut16, false>(g, M, nc, ou, ov, op16, best_next, nn, nullptr, nullptr, ctrl, sh, s); return true;
        case kFull32 * 3 + kOutNone: pass_dispatch<kFull32, kOutNone, false>(g, M, nc, ou, ov, op16, best_next, nn, nullptr, nullptr, ctrl, sh, s); return true;
        case kFull32 * 3 + kOut16: pass_dispatch<kFull32, kOut16, false>(g, M, nc, ou, ov, op16, best_next, nn, nullptr, nullptr, ctrl, sh, s); return true;
        case kFull16 * 3 + kOutNone: pass_dispatch<kFull16, kOutNone, false>(g, M, nc, ou, ov, op16, best_next, nn, nullptr, nullptr, ctrl, sh, s); return true;
        case kCompact * 3 + kOutNone: pass_dispatch<kCompact, kOutNone, false>(g, M, nc, ou, ov, op16, best_next, nn, nullptr, nullptr, ctrl, sh, s); return true;
        default: return false;
    }
}

template <int DEDUP>
static void launch_compact_flags(int in_mode, const View& g, const int32_t* M, uint64_t* flags,
                                 uint64_t* cnt, uint32_t nt, const uint64_t* dp,
                                 const uint64_t* dm, int64_t ds, hipStream_t s) {
    const dim3 gr(nt < kCompactGrid ? nt : kCompactGrid), bl(kBlock);
    switch (in_mode) {
        case kOrig: hipLaunchKernelGGL((k_compact_flags<kOrig, DEDUP>), gr, bl, 0, s, g, M, flags, cnt, nt, dp, dm, ds); break;
        case kFull32: hipLaunchKernelGGL((k_compact_flags<kFull32, DEDUP>), gr, bl, 0, s, g, M, flags, cnt, nt, dp, dm, ds); break;
        case kFull16: hipLaunchKernelGGL((k_compact_flags<kFull16, DEDUP>), gr, bl, 0, s, g, M, flags, cnt, nt, dp, dm, ds); break;
        default: hipLaunchKernelGGL((k_compact_flags<kCompact, DEDUP>), gr, bl, 0, s, g, M, flags, cnt, nt, dp, dm, ds); break;
    }
}

void launch_compact(int in_mode, const View& g, const int32_t* M, EdgeSoA out,
                    uint64_t* best_next, int64_t nn, uint64_t* flags, uint64_t* cnt,
                    uint64_t* bsum, Ctrl* ctrl, int dedup, const uint64_t* dpair,
                    const uint64_t* dmin, int64_t dslots, bool local, bool side_keys,
                    hipStream_t s) {
    if (g.len <= 0) return;
    const int sh = side_keys ? 1 : 0;
    const uint32_t nt = (uint32_t)((g.len + kRelabelTile - 1) / kRelabelTile);
    if (dedup == kDedupExact && dslots > 0)
        launch_compact_flags<kDedupExact>(in_mode, g, M, flags, cnt, nt, dpair, dmin, dslots, s);
    else if (dedup != kDedupNone && local &&
             ((int64_t)nt + kFwTiles - 1) / kFwTiles >=
                 resident_blocks(k_compact_flags_wide<kCompact>, kFwThreads)) {
        // a step for every workgroup that fits at once, else the 256-thread kernel
        const int64_t nsteps = ((int64_t)nt + kFwTiles - 1) / kFwTiles;
        const int64_t cap = resident_blocks(k_compact_flags_wide<kCompact>, kFwThreads);
        const dim3 gw((unsigned)(nsteps < cap ? nsteps : cap)), bw(kFwThreads);
        switch (in_mode) {
            case kOrig: hipLaunchKernelGGL(k_compact_flags_wide<kOrig>, gw, bw, 0, s, g, M, flags, cnt, nt); break;
            case kFull32: hipLaunchKernelGGL(k_compact_flags_wide<kFull32>, gw, bw, 0, s, g, M, flags, cnt, nt); break;
            case kFull16: hipLaunchKernelGGL(k_compact_flags_wide<kFull16>, gw, bw, 0, s, g, M, flags, cnt, nt); break;
            default: hipLaunchKernelGGL(k_compact_flags_wide<kCompact>, gw, bw, 0, s, g, M, flags, cnt, nt); break;
        }
    } else if (dedup != kDedupNone)
        launch_compact_flags<kDedupLocal>(in_mode, g, M, flags, cnt, nt, dpair, dmin, dslots, s);
    else
        launch_compact_flags<kDedupNone>(in_mode, g, M, flags, cnt, nt, dpair, dmin, dslots, s);
    launch_scan_tiles(cnt, nt, bsum, &ctrl->m_next, s);
    const int64_t nsteps = ((int64_t)nt + kSwTiles - 1) / kSwTiles;
    const int64_t cap = local ? resident_blocks(k_compact_scatter_win<kCompact>, kSwThreads) : 0;
    if (local && nsteps >= cap) {
        // a contiguous run of steps for each workgroup that fits at once (with
        // fewer steps than that the 256-thread kernel spreads the work wider)
        const int64_t per = (nsteps + cap - 1) / cap;
        const dim3 gw((unsigned)((nsteps + per - 1) / per)), bw(kSwThreads);
        switch (in_mode) {
            case kOrig: hipLaunchKernelGGL(k_compact_scatter_win<kOrig>, gw, bw, 0, s, g, M, flags, cnt, out, best_next, nt, nn, per, sh); break;
            case kFull32: hipLaunchKernelGGL(k_compact_scatter_win<kFull32>, gw, bw, 0, s, g, M, flags, cnt, out, best_next, nt, nn, per, sh); break;
            case kFull16: hipLaunchKernelGGL(k_compact_scatter_win<kFull16>, gw, bw, 0, s, g, M, flags, cnt, out, best_next, nt, nn, per, sh); break;
            default: hipLaunchKernelGGL(k_compact_scatter_win<kCompact>, gw, bw, 0, s, g, M, flags, cnt, out, best_next, nt, nn, per, sh); break;
        }
        return;
    }
    const dim3 gr(nt < kCompactGrid ? nt : kCompactGrid), bl(kBlock);
    switch (in_mode) {
        case kOrig: hipLaunchKernelGGL((k_compact_scatter<kOrig, true>), gr, bl, 0, s, g, M, flags, cnt, out, best_next, nt, sh); break;
        case kFull32: hipLaunchKernelGGL((k_compact_scatter<kFull32, true>), gr, bl, 0, s, g, M, flags, cnt, out, best_next, nt, sh); break;
        case kFull16: hipLaunchKernelGGL((k_compact_scatter<kFull16, true>), gr, bl, 0, s, g, M, flags, cnt, out, best_next, nt, sh); break;
        default: hipLaunchKernelGGL((k_compact_scatter<kCompact, true>), gr, bl, 0, s, g, M, flags, cnt, out, best_next, nt, sh); break;
    }
}

void launch_dedup_insert(int in_mode, const View& g, const int32_t* M, uint64_t* dpair,
                         uint64_t* dmin, int64_t dslots, hipStream_t s) {
    if (g.len <= 0 || dslots <= 0) return;
    const dim3 gr(grid_for(g.len, 4096)), bl(kBlock);
    auto* p = (unsigned long long*)dpair;
    auto* q = (unsigned long long*)dmin;
    switch (in_mode) {
        case kOrig: hipLaunchKernelGGL(k_dedup_insert<kOrig>, gr, bl, 0, s, g, M, p, q, dslots); break;
        case kFull32: hipLaunchKernelGGL(k_dedup_insert<kFull32>, gr, bl, 0, s, g, M, p, q, dslots); break;
        case kFull16: hipLaunchKernelGGL(k_dedup_insert<kFull16>, gr, bl, 0, s, g, M, p, q, dslots); break;
        default: hipLaunchKernelGGL(k_dedup_insert<kCompact>, gr, bl, 0, s, g, M, p, q, dslots); break;
    }
}

}  // namespace msf
