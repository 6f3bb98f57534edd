// Batched MSF: thousands of independent graphs in one persistent launch.
//
// Every graph runs all Borůvka rounds of the paper's Sec. II-C inside the
// kernel: lightest incident edge per vertex with packed (w << 32 | local edge
// index) keys, hook with the 2-cycle tie break and MSF marking, pointer
// jumping, dense relabelling of the roots, composition of the labels of the
// graph's vertices.  No host round trip is needed, so the launch can be
// captured in a hipGraph.
//
// Three lists, built by k_batch_prep in the caller's order (largest first by
// default):
//  * cooperative graphs (m >= coop_edges) are solved one at a time per XCD by
//    every workgroup running on that XCD, so the graph's per-vertex state
//    (20 B per vertex, in a global slot) stays in that XCD's L2.  The rounds
//    are cut into phases of chunks taken from an atomic ticket; the
//    workgroup that completes a phase's last chunk sets up the next phase.
//    A workgroup only ever waits for chunks that running workgroups took, so
//    nothing assumes the whole grid is resident;
//  * graphs with m <= wave_edges and n <= wave_n would be solved by one wave
//    each, all state in the wave's share of the workgroup's LDS (this tier is
//    switched off: the host never enables it, wave_n stays 0);
//  * the other graphs are solved by one workgroup each, the state in LDS when
//    n <= lds_n, else in the workgroup's own global slot.
// The lightest-edge search updates a label's minimum in one of three tiers by
// the label's degree among the edges being scanned: labels found on at least
// hot_min of a chunk's 64 sampled edge ends keep their minimum in LDS for the
// chunk (block tier); lanes of a wave sharing a label, at least wave_min of
// them, are min-reduced across the wave first (wave tier); other lanes update
// alone (thread tier).  All thresholds come from the options (autotuned).
// Every wait is bounded by wall-clock time.
#include "batch.h"
#include "prim.h"

namespace msf {

constexpr int kBatchMaxRounds = 64;
constexpr int kMaxJumps = 64;
constexpr int kEdgeIlp = 8;
constexpr uint32_t kNotReady = 0xffffffffu;       // phase id before the first set-up
constexpr uint64_t kWaitTicks = 200000000ull;     // 2 s of the 100 MHz wall clock

enum CoopKind : uint32_t {
    C_NONE = 0, C_INIT, C_MINEDGE, C_HOOK, C_JUMP, C_IDS, C_COMPOSE, C_PFILL,
    C_PBUILD, C_DONE
};

__host__ __device__ __forceinline__ int64_t tri_slot(int64_t x, int64_t y) {
    const int64_t lo = x < y ? x : y, hi = x < y ? y : x;
    return hi * (hi - 1) / 2 + lo;
}

// Inverse of tri_slot: slot s -> (lo, hi), lo < hi.
__device__ __forceinline__ void tri_pair(int64_t s, int32_t& lo, int32_t& hi) {
    int64_t h = (int64_t)((1.0 + sqrt(1.0 + 8.0 * (double)s)) * 0.5);
    while (h * (h - 1) / 2 > s) --h;
    while ((h + 1) * h / 2 <= s) ++h;
    hi = (int32_t)h;
    lo = (int32_t)(s - h * (h - 1) / 2);
}

// Ordering between workgroups of ONE XCD, which share its L2: a wave's stores
// are complete at the L2 once its vmcnt drains (the vector L1 writes through;
// every wave must drain its own before the workgroup barrier that precedes
// the signal), and a reader drops its CU's L1 before reading.  No L2
// write-back is needed, unlike the device-wide __threadfence.
__device__ __forceinline__ void xcd_release() {
    asm volatile("s_waitcnt vmcnt(0) lgkmcnt(0)" ::: "memory");
}
__device__ __forceinline__ void xcd_acquire() {
    asm volatile("buffer_inv sc1" ::: "memory");
}

__device__ __forceinline__ uint32_t xcc_id() {
    uint32_t x;
    asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID, 0, 4)" : "=s"(x));
    return x & (kMaxXcd - 1);
}

// Exclusive rank of `flag` among the workgroup's threads; *total gets the count.
template <int BS>
__device__ __forceinline__ uint32_t block_rank(bool flag, uint32_t* s_wave, uint32_t* total) {
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const uint64_t b = __ballot(flag);
    if (lane == 0) s_wave[wave] = __popcll(b);
    __syncthreads();
    uint32_t off = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < BS / kWave; ++i) {
        if (i < wave) off += s_wave[i];
        tot += s_wave[i];
    }
    __syncthreads();
    *total = tot;
    return off + lanes_below(b);
}

template <int BS>
__device__ __forceinline__ uint64_t block_sum_u64(uint64_t x, uint64_t* s_red) {
    x = wave_sum_u64(x);
    if (threadIdx.x % kWave == 0) s_red[threadIdx.x / kWave] = x;
    __syncthreads();
    uint64_t t = 0;
#pragma unroll
    for (int i = 0; i < BS / kWave; ++i) t += s_red[i];
    __syncthreads();
    return t;
}

// Thread and wave tiers of one minimum update, called by the whole wave:
// lanes sharing the first active lane's label, when at least wave_min of them
// (wave_min > 0), are min-reduced across the wave and update once; the others
// update alone.
__device__ __forceinline__ void tier_update(uint64_t* best, int32_t t, uint64_t key, bool act,
                                            int wave_min) {
    if (wave_min > 0) {
        const uint64_t am = __ballot(act);
        if (am) {
            const int leader = __builtin_ctzll(am);
            const int32_t tl = __shfl(t, leader, 64);
            const bool same = act && t == tl;
            if (__popcll(__ballot(same)) >= (wave_min > 2 ? wave_min : 2)) {
                const uint64_t k = wave_min_u64(same ? key : kKeyMax);
                if (lane_id() == leader) atomic_min_key(&best[tl], k);
                act = act && !same;
            }
        }
    }
    if (act) atomic_min_key(&best[t], key);
}

// As tier_update for lanes whose key already beat the entry as read earlier
// (a caller that issues all its reads first keeps them in flight together):
// the atomics go out without reading the entry again.
__device__ __forceinline__ void tier_commit(uint64_t* best, int32_t t, uint64_t key, bool act,
                                            int wave_min) {
    if (wave_min > 0) {
        const uint64_t am = __ballot(act);
        if (am) {
            const int leader = __builtin_ctzll(am);
            const int32_t tl = __shfl(t, leader, 64);
            const bool same = act && t == tl;
            if (__popcll(__ballot(same)) >= (wave_min > 2 ? wave_min : 2)) {
                const uint64_t k = wave_min_u64(same ? key : kKeyMax);
                if (lane_id() == leader) atomicMin((unsigned long long*)&best[tl], (unsigned long long)k);
                act = act && !same;
            }
        }
    }
    if (act) atomicMin((unsigned long long*)&best[t], (unsigned long long)key);
}

// Block tier, chosen per chunk: one wave samples 32 evenly spaced edges of
// [lo, hi) (both ends, so 64 labels) and keeps the kHot labels seen on at
// least hot_min of them; their minima live in LDS during the chunk.  Called by
// the whole workgroup (contains barriers).
template <int BS>
__device__ void chunk_hot(const int32_t* __restrict__ U, const int32_t* __restrict__ V,
                          int64_t lo, int64_t hi, int64_t n, int round, const int32_t* lab,
                          int hot_min, int32_t* s_hot, unsigned long long* s_hotmin) {
    if (threadIdx.x < kWave) {
        const int lane = threadIdx.x;
        int32_t l = -1;
        if (hi > lo) {
            const int64_t e = lo + (int64_t)(lane >> 1) * (hi - lo) / 32;
            const int32_t x = (lane & 1) ? V[e] : U[e];
            if ((uint32_t)x < (uint64_t)n) l = round == 0 ? x : lab[x];
        }
        for (int h = 0; h < kHot; ++h) {
            int best_cnt = 0;
            int32_t best_lab = -1;
            for (int i = 0; i < kWave; ++i) {
                const int32_t li = __shfl(l, i, kWave);
                const int c = __popcll(__ballot(l == li && li >= 0));
                if (c > best_cnt) { best_cnt = c; best_lab = li; }
            }
            if (lane == 0) {
                s_hot[h] = best_cnt >= hot_min ? best_lab : -1;
                s_hotmin[h] = kKeyMax;
            }
            if (best_lab >= 0 && l == best_lab) l = -1;
        }
    }
    __syncthreads();
}

// Merges the block tier's LDS minima (after the chunk; whole workgroup).
__device__ void chunk_hot_flush(uint64_t* best, const int32_t* s_hot,
                                const unsigned long long* s_hotmin) {
    __syncthreads();
    if (threadIdx.x < kHot && s_hot[threadIdx.x] >= 0 && s_hotmin[threadIdx.x] != kKeyMax)
        atomic_min_key(&best[s_hot[threadIdx.x]], s_hotmin[threadIdx.x]);
    __syncthreads();
}

// Labels whose pair table (8 B per pair), minima (8 B) and pair-label map
// (4 B) fit `bytes` of LDS: the largest p with 4 p (p - 1) + 12 p <= bytes.
__device__ __forceinline__ int64_t pair_labels(int64_t bytes) {
    int64_t p = (int64_t)sqrt((double)bytes / 4.0) + 2;
    while (p > 0 && 4 * p * (p - 1) + 12 * p > bytes) --p;
    return p;
}

// Side keys (w << 32 | edge << 1 | side) for graphs of at most 2^31 edges:
// the edge index takes 31 bits.
__device__ __forceinline__ int side_keys(int64_t m) { return m <= (1ll << 31) ? 1 : 0; }

// Lightest edge of every endpoint label over edges [lo, hi) of one graph,
// kEdgeIlp independent edges per thread (all loads and label gathers of a
// step issued before any is used).  Round 0 reads the ids directly (labels
// are the ids) and validates them.  hot (or null): the block tier's labels,
// their minima in s_hotmin; wave_min: the wave tier's threshold; sh: side
// keys (1) or w << 32 | edge (0).
template <int BS>
__device__ __forceinline__ void min_edges(const int32_t* __restrict__ U,
                                          const int32_t* __restrict__ V,
                                          const uint32_t* __restrict__ W, int64_t lo, int64_t hi,
                                          int64_t n, int round, const int32_t* lab,
                                          uint64_t* best, int& any, bool& bad,
                                          const int32_t* s_hot, unsigned long long* s_hotmin,
                                          int wave_min, int sh) {
    const int tid = threadIdx.x;
    int32_t hot[kHot];
#pragma unroll
    for (int h = 0; h < kHot; ++h) hot[h] = s_hot ? s_hot[h] : -1;
    for (int64_t base = lo; base < hi; base += (int64_t)BS * kEdgeIlp) {
        int32_t a[kEdgeIlp], b[kEdgeIlp], la[kEdgeIlp], lb[kEdgeIlp];
        uint32_t wt[kEdgeIlp];
#pragma unroll
        for (int k = 0; k < kEdgeIlp; ++k) {
            const int64_t e = base + k * BS + tid;
            a[k] = b[k] = 0;
            wt[k] = 0;
            if (e < hi) { a[k] = U[e]; b[k] = V[e]; wt[k] = W[e]; }
        }
#pragma unroll
        for (int k = 0; k < kEdgeIlp; ++k) {
            const int64_t e = base + k * BS + tid;
            la[k] = lb[k] = -1;                       // dead unless set below
            if (e >= hi || a[k] == b[k]) continue;
            if (round == 0) {
                if ((uint32_t)a[k] >= (uint64_t)n || (uint32_t)b[k] >= (uint64_t)n) {
                    bad = true;
                    continue;
                }
                la[k] = a[k];
                lb[k] = b[k];
            } else {
                la[k] = lab[a[k]];
                lb[k] = lab[b[k]];
            }
        }
        // every lane's minimum reads first, then the atomics of the keys that
        // still lower them: the reads of a lane overlap instead of running one
        // after another
        // sh = 1: side keys, the V end's key has bit 0 set (see hook_range)
        uint64_t key[kEdgeIlp], ca[kEdgeIlp], cb[kEdgeIlp];
        bool ax[kEdgeIlp], ay[kEdgeIlp];
#pragma unroll
        for (int k = 0; k < kEdgeIlp; ++k) {
            const bool act = la[k] != lb[k];
            const int64_t e = base + k * BS + tid;
            key[k] = ((uint64_t)wt[k] << 32) | ((uint64_t)e << sh);
            if (act) any = 1;
            const bool hx = act && s_hot && hot_min(hot, s_hotmin, la[k], key[k]);
            const bool hy = act && s_hot && hot_min(hot, s_hotmin, lb[k], key[k] | (uint64_t)sh);
            ax[k] = act && !hx;
            ay[k] = act && !hy;
            ca[k] = ax[k] ? best[la[k]] : 0;
            cb[k] = ay[k] ? best[lb[k]] : 0;
        }
#pragma unroll
        for (int k = 0; k < kEdgeIlp; ++k) {
            const uint64_t kb = key[k] | (uint64_t)sh;
            tier_commit(best, la[k], key[k], ax[k] && key[k] < ca[k], wave_min);
            tier_commit(best, lb[k], kb, ay[k] && kb < cb[k], wave_min);
        }
    }
}

// The per-vertex steps below take kVtxIlp vertices per thread at a time and
// issue each level of their dependent loads together (a lane's chains overlap
// instead of running one after another).
constexpr int kVtxIlp = 4;

// Hook + MSF mark over labels [lo, hi): parent = other end of the lightest
// edge; of a 2-cycle (same edge chosen by both) the smaller label is the root.
// sh = 1: side keys (w << 32 | edge << 1 | side, side 1 when the label is
// the edge's V end), so only the other end is read and mapped, and the other
// end's key for the same edge has the side bit flipped; sh = 0: w << 32 |
// edge, both ends read.  *roots counts the roots that found an edge (the
// next round's labels).
__device__ __forceinline__ uint64_t hook_range(const int32_t* __restrict__ U,
                                               const int32_t* __restrict__ V, int64_t lo,
                                               int64_t hi, int stride, const int32_t* lab,
                                               const uint64_t* best, int32_t* par,
                                               uint8_t* mask, int sh, uint32_t* roots) {
    uint64_t wsum = 0;
    for (int64_t x0 = lo + threadIdx.x; x0 < hi; x0 += (int64_t)stride * kVtxIlp) {
        uint64_t b[kVtxIlp], bo[kVtxIlp];
        int32_t la[kVtxIlp], lb[kVtxIlp], other[kVtxIlp];
#pragma unroll
        for (int k = 0; k < kVtxIlp; ++k) {
            const int64_t x = x0 + (int64_t)k * stride;
            b[k] = x < hi ? best[x] : kKeyMax;
        }
        if (sh) {
#pragma unroll
            for (int k = 0; k < kVtxIlp; ++k) {
                const uint32_t pos = (uint32_t)b[k] >> 1;
                la[k] = b[k] != kKeyMax ? ((b[k] & 1u) ? U[pos] : V[pos]) : 0;
            }
#pragma unroll
            for (int k = 0; k < kVtxIlp; ++k) other[k] = b[k] != kKeyMax ? lab[la[k]] : 0;
        } else {
#pragma unroll
            for (int k = 0; k < kVtxIlp; ++k) {
                const uint32_t pos = (uint32_t)b[k];
                la[k] = b[k] != kKeyMax ? U[pos] : 0;
                lb[k] = b[k] != kKeyMax ? V[pos] : 0;
            }
#pragma unroll
            for (int k = 0; k < kVtxIlp; ++k) {
                la[k] = b[k] != kKeyMax ? lab[la[k]] : 0;
                lb[k] = b[k] != kKeyMax ? lab[lb[k]] : 0;
            }
#pragma unroll
            for (int k = 0; k < kVtxIlp; ++k) {
                const int64_t x = x0 + (int64_t)k * stride;
                other[k] = la[k] == (int32_t)x ? lb[k] : la[k];
            }
        }
#pragma unroll
        for (int k = 0; k < kVtxIlp; ++k) bo[k] = b[k] != kKeyMax ? best[other[k]] : 0;
#pragma unroll
        for (int k = 0; k < kVtxIlp; ++k) {
            const int64_t x = x0 + (int64_t)k * stride;
            if (x >= hi) continue;
            if (b[k] == kKeyMax || (bo[k] == (b[k] ^ (uint64_t)sh) && (int32_t)x < other[k])) {
                par[x] = (int32_t)x;
                if (b[k] != kKeyMax) ++*roots;
            } else {
                par[x] = other[k];
                mask[(uint32_t)b[k] >> sh] = 1;
                wsum += b[k] >> 32;
            }
        }
    }
    return wsum;
}

// Pointer jumping over [lo, hi): each vertex walks up its parent chain, at
// most kWalkSteps steps, and keeps the furthest vertex reached as its
// parent (the root when the walk ends there).  Parents only ever move towards
// the root, so reading entries that others update meanwhile is harmless.
// True if some walk stopped short of its root (another pass is needed).
constexpr int kWalkSteps = 32;
__device__ __forceinline__ bool jump_range(int32_t* par, int64_t lo, int64_t hi, int stride) {
    bool cut = false;
    for (int64_t x0 = lo + threadIdx.x; x0 < hi; x0 += (int64_t)stride * kVtxIlp) {
        int32_t p[kVtxIlp], p0[kVtxIlp];
        bool walk[kVtxIlp];
#pragma unroll
        for (int k = 0; k < kVtxIlp; ++k) {
            const int64_t x = x0 + (int64_t)k * stride;
            p[k] = x < hi ? par[x] : 0;
            p0[k] = p[k];
            walk[k] = x < hi && p[k] != (int32_t)x;
        }
        for (int step = 0; step < kWalkSteps; ++step) {   // the lane's walks in lockstep
            int32_t pp[kVtxIlp];
            bool more = false;
#pragma unroll
            for (int k = 0; k < kVtxIlp; ++k) pp[k] = walk[k] ? par[p[k]] : p[k];
#pragma unroll
            for (int k = 0; k < kVtxIlp; ++k) {
                if (!walk[k]) continue;
                if (pp[k] == p[k]) {
                    walk[k] = false;                       // p[k] is the root
                } else {
                    p[k] = pp[k];
                    more = true;
                }
            }
            if (!more) break;
        }
#pragma unroll
        for (int k = 0; k < kVtxIlp; ++k) {
            const int64_t x = x0 + (int64_t)k * stride;
            if (x < hi && p[k] != p0[k]) par[x] = p[k];
            if (walk[k]) cut = true;
        }
    }
    return cut;
}

// Label composition over [lo, hi): each label becomes nid of its component's
// root, the new id (the ids pass gives a root whose component found no edge
// nid -1: that label is done).
__device__ __forceinline__ void compose_range(int32_t* lab, const int32_t* par,
                                              const int32_t* nid, int64_t lo, int64_t hi,
                                              int stride) {
    for (int64_t i0 = lo + threadIdx.x; i0 < hi; i0 += (int64_t)stride * kVtxIlp) {
        int32_t l[kVtxIlp], r[kVtxIlp];
#pragma unroll
        for (int k = 0; k < kVtxIlp; ++k) {
            const int64_t i = i0 + (int64_t)k * stride;
            l[k] = i < hi ? lab[i] : -1;
        }
#pragma unroll
        for (int k = 0; k < kVtxIlp; ++k) r[k] = l[k] >= 0 ? par[l[k]] : 0;
#pragma unroll
        for (int k = 0; k < kVtxIlp; ++k) r[k] = l[k] >= 0 ? nid[r[k]] : -1;
#pragma unroll
        for (int k = 0; k < kVtxIlp; ++k) {
            const int64_t i = i0 + (int64_t)k * stride;
            if (i < hi && l[k] >= 0) lab[i] = r[k];
        }
    }
}

// --------------------------------------------------- one workgroup per graph

// State arrays of `cap` vertices (LDS or a global slot).
// tiers: the state is in global memory (the slot), so the block and wave
// tiers of the lightest-edge search apply; in LDS every update is cheap.
// pair_lds (or null), pair_bytes: LDS the state does not use.  Once at most
// pair_labels(pair_bytes) labels are left and their pairs are fewer than half
// the edges, the edges are reduced to the lightest edge of each label pair
// (a triangular table in that LDS) and the remaining rounds scan the table.
template <int BS>
__device__ void solve_graph(const BatchArgs& A, int64_t g, int64_t cap, int32_t* lab,
                            uint64_t* best, int32_t* par, int32_t* nid, uint32_t* s_wave,
                            bool tiers, int32_t* s_hot, unsigned long long* s_hotmin,
                            unsigned long long* pair_lds, int64_t pair_bytes) {
    const int tid = threadIdx.x;
    const int64_t e0 = A.eoff[g];
    const int64_t m = A.eoff[g + 1] - e0;
    const int64_t n = A.voff[g + 1] - A.voff[g];
    const int32_t* U = A.u + e0;
    const int32_t* V = A.v + e0;
    const uint32_t* W = A.w + e0;
    uint8_t* mask = A.mask + e0;
    if (tid == 0 && A.ticks) A.ticks[A.G + 1 + g] = wall_clock64();
    const bool bad_shape = n < 0 || n > cap || m < 0 || m > 0xffffffffLL;
    bool bad = bad_shape;
    uint64_t wsum = 0;
    const int sh = side_keys(m);
    const int64_t pmax = pair_lds ? pair_labels(pair_bytes) : 0;
    int64_t pn = 0;                          // > 0: the rounds scan the pair table of pn labels
    unsigned long long* pbest = nullptr;     // pair rounds: this round's minima, in LDS
    int32_t* plab = nullptr;                 // pair-table label -> current label
    if (!bad_shape) {
        for (int64_t i = tid; i < m; i += BS) mask[i] = 0;
        for (int64_t x = tid; x < n; x += BS) {
            lab[x] = (int32_t)x;
            best[x] = kKeyMax;
        }
        int64_t ncur = n;
        __syncthreads();
        for (int round = 0; round < kBatchMaxRounds && ncur > 1; ++round) {
            int any = 0;
            if (pn) {                        // minima over the pair table, in LDS
                for (int64_t x = tid; x < ncur; x += BS) pbest[x] = kKeyMax;
                __syncthreads();
                const int64_t np = pn * (pn - 1) / 2;
                for (int64_t s = tid; s < np; s += BS) {
                    const uint64_t key = pair_lds[s];
                    if (key == kKeyMax) continue;
                    int32_t lo, hi;
                    tri_pair(s, lo, hi);
                    const int32_t lx = plab[lo], ly = plab[hi];
                    if (lx == ly) continue;
                    any = 1;
                    if (key < pbest[lx]) atomicMin(&pbest[lx], (unsigned long long)key);
                    if (key < pbest[ly]) atomicMin(&pbest[ly], (unsigned long long)key);
                }
                __syncthreads();
                for (int64_t x = tid; x < ncur; x += BS) best[x] = pbest[x];
            } else {
                const bool block_tier = tiers && A.hot_min > 0;
                if (block_tier)
                    chunk_hot<BS>(U, V, 0, m, n, round, lab, A.hot_min, s_hot, s_hotmin);
                min_edges<BS>(U, V, W, 0, m, n, round, lab, best, any, bad,
                              block_tier ? s_hot : nullptr, s_hotmin, tiers ? A.wave_min : 0,
                              sh);
                if (block_tier) chunk_hot_flush(best, s_hot, s_hotmin);
            }
            if (!__syncthreads_or(any) || __syncthreads_or(bad)) break;
            uint32_t nroot_unused = 0;   // the pair table's keys (w << 32 | edge) carry no side
            wsum += hook_range(U, V, 0, ncur, BS, lab, best, par, mask, pn ? 0 : sh,
                               &nroot_unused);
            __syncthreads();
            for (int it = 0; it < kMaxJumps; ++it) {                   // pointer jumping
                const int changed = jump_range(par, 0, ncur, BS) ? 1 : 0;
                if (!__syncthreads_or(changed)) break;
            }
            int64_t roots = 0;                                         // dense ids of roots
            for (int64_t base = 0; base < ncur; base += BS) {
                const int64_t x = base + tid;
                const bool self = x < ncur && par[x] == (int32_t)x;
                const bool r = self && best[x] != kKeyMax;
                uint32_t tot;
                const uint32_t rk = block_rank<BS>(r, s_wave, &tot);
                if (r) nid[x] = (int32_t)(roots + rk);
                else if (self) nid[x] = -1;                             // no edge: done
                roots += tot;
            }
            __syncthreads();
            compose_range(lab, par, nid, 0, n, BS);                    // compose labels
            if (pn) compose_range(plab, par, nid, 0, pn, BS);
            for (int64_t x = tid; x < roots; x += BS) best[x] = kKeyMax;   // next round
            ncur = roots;
            __syncthreads();
            if (!pn && ncur >= 2 && ncur <= pmax && ncur * (ncur - 1) / 2 < m / 2) {
                // the lightest edge of each pair of the ncur labels; pair-table
                // label i is label i now
                pn = ncur;
                const int64_t np = pn * (pn - 1) / 2;
                pbest = pair_lds + np;
                plab = reinterpret_cast<int32_t*>(pbest + pn);
                for (int64_t s = tid; s < np; s += BS) pair_lds[s] = kKeyMax;
                for (int64_t i = tid; i < pn; i += BS) plab[i] = (int32_t)i;
                __syncthreads();
                for (int64_t e = tid; e < m; e += BS) {
                    const int32_t a = U[e], b = V[e];
                    if (a == b) continue;
                    const int32_t la = lab[a], lb = lab[b];
                    if (la == lb || la < 0 || lb < 0) continue;
                    const uint64_t key = ((uint64_t)W[e] << 32) | (uint64_t)e;
                    unsigned long long* p = &pair_lds[tri_slot(la, lb)];
                    if (key < *p) atomicMin(p, (unsigned long long)key);
                }
                __syncthreads();
            }
        }
    }
    wsum = wave_sum_u64(wsum);
    __shared__ unsigned long long s_total;
    if (tid == 0) s_total = 0;
    __syncthreads();
    if (lane_id() == 0 && wsum) atomicAdd(&s_total, (unsigned long long)wsum);
    const int anybad = __syncthreads_or(bad);
    if (tid == 0) {
        A.totals[g] = anybad ? kKeyMax : (uint64_t)s_total;
        if (A.ticks) A.ticks[g] = wall_clock64();
    }
    __syncthreads();
}

// ------------------------------------------------------- one wave per graph

// Orders the wave's LDS accesses: every lane's earlier LDS operations have
// completed before any lane goes on.
__device__ __forceinline__ void wave_sync() {
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    __builtin_amdgcn_wave_barrier();
}

// The whole of one small graph by one wave, its state (20 B per vertex) in
// the wave's share of LDS: the rounds of solve_graph with wave-wide votes
// instead of workgroup barriers.
__device__ void solve_graph_wave(const BatchArgs& A, int64_t g, int64_t cap, int32_t* lab,
                                 uint64_t* best, int32_t* par, int32_t* nid) {
    const int lane = lane_id();
    const int64_t e0 = A.eoff[g];
    const int64_t m = A.eoff[g + 1] - e0;
    const int64_t n = A.voff[g + 1] - A.voff[g];
    const int32_t* U = A.u + e0;
    const int32_t* V = A.v + e0;
    const uint32_t* W = A.w + e0;
    uint8_t* mask = A.mask + e0;
    if (lane == 0 && A.ticks) A.ticks[A.G + 1 + g] = wall_clock64();
    const bool bad_shape = n < 0 || n > cap || m < 0 || m > 0xffffffffLL;
    bool bad = bad_shape;
    uint64_t wsum = 0;
    if (!bad_shape) {
        for (int64_t i = lane; i < m; i += kWave) mask[i] = 0;
        for (int64_t x = lane; x < n; x += kWave) lab[x] = (int32_t)x;
        int64_t ncur = n;
        wave_sync();
        for (int round = 0; round < kBatchMaxRounds && ncur > 1; ++round) {
            for (int64_t x = lane; x < ncur; x += kWave) best[x] = kKeyMax;
            wave_sync();
            bool any = false;
            for (int64_t e = lane; e < m; e += kWave) {
                int32_t a = U[e], b = V[e];
                if (a == b) continue;
                if (round == 0) {
                    if ((uint32_t)a >= (uint64_t)n || (uint32_t)b >= (uint64_t)n) {
                        bad = true;
                        continue;
                    }
                } else {
                    a = lab[a];
                    b = lab[b];
                    if (a == b) continue;
                }
                any = true;
                const uint64_t key = ((uint64_t)W[e] << 32) | (uint64_t)e;
                atomic_min_key(&best[a], key);
                atomic_min_key(&best[b], key);
            }
            wave_sync();
            if (!__ballot(any) || __ballot(bad)) break;
            for (int64_t x = lane; x < ncur; x += kWave) {      // hook + MSF mark
                const uint64_t b = best[x];
                if (b == kKeyMax) { par[x] = (int32_t)x; continue; }
                const uint32_t pos = (uint32_t)b;
                const int32_t la = round == 0 ? U[pos] : lab[U[pos]];
                const int32_t lb = round == 0 ? V[pos] : lab[V[pos]];
                const int32_t other = la == (int32_t)x ? lb : la;
                if (best[other] == b && (int32_t)x < other) {
                    par[x] = (int32_t)x;
                } else {
                    par[x] = other;
                    mask[pos] = 1;
                    wsum += b >> 32;
                }
            }
            wave_sync();
            for (int it = 0; it < kMaxJumps; ++it) {             // pointer jumping
                bool changed = false;
                for (int64_t x = lane; x < ncur; x += kWave) {
                    const int32_t p = par[x], pp = par[p];
                    if (p != pp) { par[x] = pp; changed = true; }
                }
                wave_sync();
                if (!__ballot(changed)) break;
            }
            int64_t roots = 0;                                   // dense ids of roots
            for (int64_t base = 0; base < ncur; base += kWave) {
                const int64_t x = base + lane;
                const bool r = x < ncur && par[x] == (int32_t)x && best[x] != kKeyMax;
                const uint64_t bal = __ballot(r);
                if (r) nid[x] = (int32_t)(roots + lanes_below(bal));
                roots += __popcll(bal);
            }
            wave_sync();
            for (int64_t i = lane; i < n; i += kWave) {          // compose labels
                const int32_t l = lab[i];
                if (l >= 0) lab[i] = best[l] == kKeyMax ? -1 : nid[par[l]];
            }
            ncur = roots;
            wave_sync();
        }
    }
    wsum = wave_sum_u64(wsum);
    const bool anybad = __ballot(bad) != 0;
    if (lane == 0) {
        A.totals[g] = anybad ? kKeyMax : wsum;
        if (A.ticks) A.ticks[g] = wall_clock64();
    }
}

// ------------------------------------------------- cooperative (one per XCD)

struct SlotView {
    uint64_t* best;
    int32_t* lab;
    int32_t* par;
    int32_t* nid;
    uint32_t* cnt;     // roots per vertex chunk, then their exclusive prefix
    uint64_t* pairs;   // cooperative slots: lightest key per vertex pair
    int32_t* plab;     // cooperative slots: current label of each pair-table vertex
};

__device__ __forceinline__ SlotView slot_view(char* slot, int64_t nmax, size_t slot_bytes) {
    SlotView s;
    const size_t cap = (size_t)nmax;
    s.best = reinterpret_cast<uint64_t*>(slot);
    s.lab = reinterpret_cast<int32_t*>(slot + cap * 8);
    s.par = s.lab + cap;
    s.nid = s.par + cap;
    s.cnt = reinterpret_cast<uint32_t*>(s.nid + cap);
    s.pairs = reinterpret_cast<uint64_t*>(slot + slot_bytes);
    s.plab = reinterpret_cast<int32_t*>(s.pairs + kPairMax * (kPairMax - 1) / 2);
    return s;
}

__device__ __forceinline__ uint32_t chunks_of(int64_t len, int64_t per) {
    return (uint32_t)((len + per - 1) / per);
}

// Publishes phase p (thread 0 of the workgroup that completed phase p - 1).
__device__ void coop_setup(XcdWork* X, uint32_t p, uint32_t kind, uint32_t nchunks) {
    X->kind[p & 1] = kind;
    X->nchunks[p & 1] = nchunks;
    X->done[p & 1] = 0;
    xcd_release();
    atomicExch((unsigned long long*)&X->ticket, (unsigned long long)((uint64_t)p << 32));
}

// Takes the next cooperative graph (or finishes) and publishes phase p.
template <int BS>
__device__ void coop_next_graph(const BatchArgs& A, XcdWork* X, uint32_t p) {
    constexpr int64_t CV = (int64_t)BS * kCoopVertsPerThread;
    constexpr int64_t CE = (int64_t)BS * kCoopEdgesPerThread;
    while (true) {
        const uint32_t gi = atomicAdd(&A.q->big_next, 1u);
        if (gi >= A.q->nbig) {
            coop_setup(X, p, C_DONE, 0);
            return;
        }
        const int64_t g = A.big[gi];
        const int64_t m = A.eoff[g + 1] - A.eoff[g];
        const int64_t n = A.voff[g + 1] - A.voff[g];
        if (A.ticks) A.ticks[A.G + 1 + g] = wall_clock64();
        if (n < 0 || n > A.nmax || m < 0 || m > 0xffffffffLL) {
            A.totals[g] = kKeyMax;
            if (A.ticks) A.ticks[g] = wall_clock64();
            continue;
        }
        X->graph = g;
        X->n = n;
        X->m = m;
        X->ncur = n;
        X->round = 0;
        X->total = 0;
        X->pair_mode = 0;
        X->pn = 0;
        X->f_any = X->f_bad = X->f_changed = 0;
        const uint32_t ce = chunks_of(m, CE), cv = chunks_of(n, CV);
        coop_setup(X, p, C_INIT, ce > cv ? ce : cv);
        return;
    }
}

template <int BS>
__device__ void coop_finish(const BatchArgs& A, XcdWork* X, uint32_t p, bool bad) {
    const int64_t g = X->graph;
    A.totals[g] = (bad || A.q->err) ? kKeyMax : X->total;
    if (A.ticks) A.ticks[g] = wall_clock64();
    coop_next_graph<BS>(A, X, p);
}

// Sets up phase p + 1 after phase p (of kind `kind`) completed.
template <int BS>
__device__ void coop_transition(const BatchArgs& A, XcdWork* X, const SlotView& S, uint32_t p,
                                uint32_t kind) {
    constexpr int64_t CV = (int64_t)BS * kCoopVertsPerThread;
    constexpr int64_t CE = (int64_t)BS * kCoopEdgesPerThread;
    constexpr int64_t CP = (int64_t)BS * kCoopPairsPerThread;
    const uint32_t q = p + 1;
    switch (kind) {
        case C_INIT:
            if (X->ncur <= 1 || X->m == 0) coop_finish<BS>(A, X, q, false);
            else coop_setup(X, q, C_MINEDGE, chunks_of(X->m, CE));
            break;
        case C_MINEDGE: {
            const uint32_t any = X->f_any, bad = X->f_bad;
            X->f_any = 0;
            if (bad || !any) coop_finish<BS>(A, X, q, bad != 0);
            else coop_setup(X, q, C_HOOK, chunks_of(X->ncur, CV));
            break;
        }
        case C_HOOK:
            X->jit = 0;
            X->f_changed = 0;
            coop_setup(X, q, C_JUMP, chunks_of(X->ncur, CV));
            break;
        case C_JUMP: {
            const uint32_t changed = X->f_changed;
            X->f_changed = 0;
            if (changed && ++X->jit < (uint32_t)kMaxJumps) {
                coop_setup(X, q, C_JUMP, chunks_of(X->ncur, CV));
                break;
            }
            // the roots counted per chunk by the hook phase: their exclusive
            // prefix, the first id of each chunk's roots
            const uint32_t nch = chunks_of(X->ncur, CV);
            uint64_t sum = 0;
            for (uint32_t c = 0; c < nch; ++c) {
                const uint32_t v = S.cnt[c];
                S.cnt[c] = (uint32_t)sum;
                sum += v;
            }
            X->nnext = (int64_t)sum;
            coop_setup(X, q, C_IDS, nch);
            break;
        }
        case C_IDS: {
            const uint32_t cn = chunks_of(X->n, CV), cp = chunks_of(X->pn, CV);
            coop_setup(X, q, C_COMPOSE, cn > cp ? cn : cp);
            break;
        }
        case C_COMPOSE:   // the compose phase also cleared the next round's minima
            X->ncur = X->nnext;
            X->round += 1;
            if (X->ncur <= 1 || X->round >= (uint32_t)kBatchMaxRounds) {
                coop_finish<BS>(A, X, q, false);
            } else if (!X->pair_mode && X->ncur <= kPairMax &&
                       X->ncur * (X->ncur - 1) / 2 < X->m / 2) {
                X->pn = X->ncur;
                const uint32_t cs = chunks_of(X->pn * (X->pn - 1) / 2, CP);
                const uint32_t cv = chunks_of(X->pn, CV);
                coop_setup(X, q, C_PFILL, cs > cv ? cs : cv);
            } else if (X->pair_mode) {
                coop_setup(X, q, C_MINEDGE, chunks_of(X->pn * (X->pn - 1) / 2, CP));
            } else {
                coop_setup(X, q, C_MINEDGE, chunks_of(X->m, CE));
            }
            break;
        case C_PFILL:
            coop_setup(X, q, C_PBUILD, chunks_of(X->m, CE));
            break;
        case C_PBUILD:
            X->pair_mode = 1;
            coop_setup(X, q, C_MINEDGE, chunks_of(X->pn * (X->pn - 1) / 2, CP));
            break;
        default:
            break;
    }
}

struct CoopParams {
    int64_t g, n, m, ncur, nnext, e0, pn;
    uint32_t kind, nchunks, round, pair_mode;
};

// One chunk of a phase, by the whole workgroup.
template <int BS>
__device__ void coop_chunk(const BatchArgs& A, XcdWork* X, const SlotView& S,
                           const CoopParams& P, uint32_t chunk, uint32_t* s_wave,
                           uint64_t* s_red, int32_t* s_hot, unsigned long long* s_hotmin) {
    constexpr int64_t CV = (int64_t)BS * kCoopVertsPerThread;
    constexpr int64_t CE = (int64_t)BS * kCoopEdgesPerThread;
    constexpr int64_t CP = (int64_t)BS * kCoopPairsPerThread;
    const int tid = threadIdx.x;
    const int32_t* U = A.u + P.e0;
    const int32_t* V = A.v + P.e0;
    const uint32_t* W = A.w + P.e0;
    uint8_t* mask = A.mask + P.e0;
    const int64_t v0 = (int64_t)chunk * CV, e0 = (int64_t)chunk * CE;
    const int64_t vn = v0 + CV < P.ncur ? v0 + CV : P.ncur;    // vertex chunk end (live labels)
    switch (P.kind) {
        case C_INIT: {
            const int64_t eh = e0 + CE < P.m ? e0 + CE : P.m;
            for (int64_t i = e0 + tid; i < eh; i += BS) mask[i] = 0;
            const int64_t xh = v0 + CV < P.n ? v0 + CV : P.n;
            for (int64_t x = v0 + tid; x < xh; x += BS) {
                S.lab[x] = (int32_t)x;
                S.best[x] = kKeyMax;
            }
            break;
        }
        case C_MINEDGE: {
            int any = 0;
            bool bad = false;
            if (P.pair_mode) {            // over the pair table
                const int64_t np = P.pn * (P.pn - 1) / 2;
                const int64_t s0 = (int64_t)chunk * CP, sh = s0 + CP < np ? s0 + CP : np;
                for (int64_t base = s0; base < sh; base += BS) {   // uniform per wave
                    const int64_t sl = base + tid;
                    const uint64_t key = sl < sh ? S.pairs[sl] : kKeyMax;
                    int32_t lx = -1, ly = -1;
                    if (key != kKeyMax) {
                        int32_t lo, hi;
                        tri_pair(sl, lo, hi);
                        lx = S.plab[lo];
                        ly = S.plab[hi];
                    }
                    const bool act = lx != ly;
                    if (act) any = 1;
                    tier_update(S.best, lx, key, act, A.wave_min);
                    tier_update(S.best, ly, key, act, A.wave_min);
                }
            } else {
                const int64_t eh = e0 + CE < P.m ? e0 + CE : P.m;
                const bool block_tier = A.hot_min > 0;
                if (block_tier)
                    chunk_hot<BS>(U, V, e0, eh, P.n, (int)P.round, S.lab, A.hot_min, s_hot,
                                  s_hotmin);
                min_edges<BS>(U, V, W, e0, eh, P.n, (int)P.round, S.lab, S.best, any, bad,
                              block_tier ? s_hot : nullptr, s_hotmin, A.wave_min,
                              side_keys(P.m));
                if (block_tier) chunk_hot_flush(S.best, s_hot, s_hotmin);
            }
            const int bany = __syncthreads_or(any), bbad = __syncthreads_or(bad);
            if (tid == 0) {
                if (bany) atomicOr(&X->f_any, 1u);
                if (bbad) atomicOr(&X->f_bad, 1u);
            }
            break;
        }
        case C_HOOK: {   // also counts the chunk's roots (jumping leaves roots as they are)
            // the pair table's keys (w << 32 | edge) carry no side
            uint32_t nr = 0;
            const uint64_t ws = block_sum_u64<BS>(
                hook_range(U, V, v0, vn, BS, S.lab, S.best, S.par, mask,
                           P.pair_mode ? 0 : side_keys(P.m), &nr),
                s_red);
            const uint64_t rc = block_sum_u64<BS>(nr, s_red);
            if (tid == 0) {
                if (ws) atomicAdd((unsigned long long*)&X->total, (unsigned long long)ws);
                S.cnt[chunk] = (uint32_t)rc;
            }
            break;
        }
        case C_JUMP: {
            const int changed = jump_range(S.par, v0, vn, BS) ? 1 : 0;
            if (__syncthreads_or(changed) && tid == 0) atomicOr(&X->f_changed, 1u);
            break;
        }
        case C_IDS: {
            int64_t roots = S.cnt[chunk];
            for (int64_t base = v0; base < v0 + CV; base += BS) {
                const int64_t x = base + tid;
                const bool self = x < vn && S.par[x] == (int32_t)x;
                const bool rt = self && S.best[x] != kKeyMax;
                uint32_t tot;
                const uint32_t rk = block_rank<BS>(rt, s_wave, &tot);
                if (rt) S.nid[x] = (int32_t)(roots + rk);
                else if (self) S.nid[x] = -1;           // no edge: its labels are done
                roots += tot;
            }
            break;
        }
        case C_COMPOSE: {   // compose reads no minimum: the next round's are cleared here
            const int64_t xh = v0 + CV < P.n ? v0 + CV : P.n;
            compose_range(S.lab, S.par, S.nid, v0, xh, BS);
            const int64_t bh = v0 + CV < P.nnext ? v0 + CV : P.nnext;
            for (int64_t x = v0 + tid; x < bh; x += BS) S.best[x] = kKeyMax;
            if (P.pair_mode) {
                const int64_t ph = v0 + CV < P.pn ? v0 + CV : P.pn;
                compose_range(S.plab, S.par, S.nid, v0, ph, BS);
            }
            break;
        }
        case C_PFILL: {                   // empty pair table; pair vertex i = label i
            const int64_t np = P.pn * (P.pn - 1) / 2;
            const int64_t s0 = (int64_t)chunk * CP, sh = s0 + CP < np ? s0 + CP : np;
            for (int64_t sl = s0 + tid; sl < sh; sl += BS) S.pairs[sl] = kKeyMax;
            const int64_t ph = v0 + CV < P.pn ? v0 + CV : P.pn;
            for (int64_t i = v0 + tid; i < ph; i += BS) S.plab[i] = (int32_t)i;
            break;
        }
        case C_PBUILD: {                  // lightest edge per pair of current labels
            const int64_t eh = e0 + CE < P.m ? e0 + CE : P.m;
            for (int64_t e = e0 + tid; e < eh; e += BS) {
                const int32_t a = U[e], b = V[e];
                if (a == b) continue;
                const int32_t la = S.lab[a], lb = S.lab[b];
                if (la == lb || la < 0 || lb < 0) continue;
                atomic_min_key(&S.pairs[tri_slot(la, lb)], ((uint64_t)W[e] << 32) | (uint64_t)e);
            }
            break;
        }
        default:
            break;
    }
}

// Waits (thread 0) until the ticket leaves phase p; false after kWaitTicks.
__device__ bool coop_wait(XcdWork* X, uint32_t p, BatchQueue* q) {
    const uint64_t deadline = wall_clock64() + kWaitTicks;
    uint32_t nap = 1;
    while ((uint32_t)(__hip_atomic_load(&X->ticket, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >>
                      32) == p) {
        if (wall_clock64() > deadline ||
            __hip_atomic_load(&q->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
            atomicOr(&q->err, 1u);
            return false;
        }
        if (nap == 1) __builtin_amdgcn_s_sleep(1);
        else if (nap == 2) __builtin_amdgcn_s_sleep(4);
        else __builtin_amdgcn_s_sleep(16);
        nap = nap < 3 ? nap + 1 : 3;
    }
    return true;
}

template <int BS>
__device__ void coop_run(const BatchArgs& A, uint32_t* s_wave, uint64_t* s_red, int32_t* s_hot,
                         unsigned long long* s_hotmin) {
    __shared__ uint64_t s_ticket;
    __shared__ CoopParams s_p;
    __shared__ uint32_t s_flag;
    const uint32_t xcd = xcc_id();
    XcdWork* X = &A.xw[xcd];
    const SlotView S = slot_view(A.xslots + (size_t)xcd * A.xslot_bytes, A.nmax, A.slot_bytes);
    if (threadIdx.x == 0 && atomicCAS(&X->state, 0u, 1u) == 0u) {
        __threadfence();
        coop_next_graph<BS>(A, X, 0);        // the first workgroup here starts phase 0
    }
    while (true) {
        if (threadIdx.x == 0) {
            const uint64_t t = __hip_atomic_fetch_add(&X->ticket, (uint64_t)1, __ATOMIC_RELAXED,
                                                      __HIP_MEMORY_SCOPE_AGENT);
            s_ticket = t;
            const uint32_t p = (uint32_t)(t >> 32);
            s_flag = 0;
            if (p != kNotReady) {
                xcd_acquire();
                s_p.kind = X->kind[p & 1];
                s_p.nchunks = X->nchunks[p & 1];
                s_p.g = X->graph;
                s_p.n = X->n;
                s_p.m = X->m;
                s_p.ncur = X->ncur;
                s_p.nnext = X->nnext;
                s_p.round = X->round;
                s_p.pn = X->pn;
                s_p.pair_mode = X->pair_mode;
                s_p.e0 = s_p.kind == C_DONE ? 0 : A.eoff[s_p.g];
            }
        }
        __syncthreads();
        const uint64_t t = s_ticket;
        const uint32_t p = (uint32_t)(t >> 32), chunk = (uint32_t)t;
        const CoopParams P = s_p;
        __syncthreads();
        if (p != kNotReady && P.kind == C_DONE) break;
        if (p == kNotReady || chunk >= P.nchunks) {       // nothing left here: wait
            if (threadIdx.x == 0) s_flag = coop_wait(X, p, A.q) ? 0u : 1u;
            __syncthreads();
            const uint32_t gave_up = s_flag;
            __syncthreads();
            if (gave_up) break;
            continue;
        }
        coop_chunk<BS>(A, X, S, P, chunk, s_wave, s_red, s_hot, s_hotmin);
        xcd_release();                       // every wave's stores reach the L2 ...
        __syncthreads();
        if (threadIdx.x == 0) {              // ... before the chunk counts as done
            const uint32_t d = atomicAdd(&X->done[p & 1], 1u);
            if (d + 1 == P.nchunks) {
                xcd_acquire();
                coop_transition<BS>(A, X, S, p, P.kind);
            }
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------ kernels

template <int BS>
__global__ __launch_bounds__(BS) void k_batch(BatchArgs A) {
    extern __shared__ uint64_t lds[];
    __shared__ uint32_t s_wave[BS / kWave];
    __shared__ uint64_t s_red[BS / kWave];
    __shared__ int64_t s_g;
    __shared__ int32_t s_hot[kHot];
    __shared__ unsigned long long s_hotmin[kHot];
    if (threadIdx.x == 0 && A.ticks)
        atomicMin((unsigned long long*)&A.ticks[A.G], (unsigned long long)wall_clock64());
    if (__hip_atomic_load(&A.q->nbig, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) > 0)
        coop_run<BS>(A, s_wave, s_red, s_hot, s_hotmin);

    const int64_t nsmall = (int64_t)A.q->nsmall;
    const int64_t cap = A.lds_n;
    char* wslot = A.wslots + (size_t)blockIdx.x * A.slot_bytes;
    const SlotView G = slot_view(wslot, A.nmax, A.slot_bytes);
    while (true) {
        if (threadIdx.x == 0) s_g = (int64_t)atomicAdd(&A.q->small_next, 1u);
        __syncthreads();
        const int64_t gi = s_g;
        __syncthreads();
        if (gi >= nsmall) break;
        const int64_t g = A.small[gi];
        if (A.voff[g + 1] - A.voff[g] <= cap) {
            int32_t* lab = reinterpret_cast<int32_t*>(lds + cap);
            solve_graph<BS>(A, g, cap, lab, lds, lab + cap, lab + 2 * cap, s_wave, false, s_hot,
                            s_hotmin, nullptr, 0);
        } else {   // the state is in the slot: the LDS holds the pair table
            solve_graph<BS>(A, g, A.nmax, G.lab, G.best, G.par, G.nid, s_wave, true, s_hot,
                            s_hotmin, reinterpret_cast<unsigned long long*>(lds), cap * 20);
        }
    }

    // Wave graphs: from here on every wave works alone, on its share of the
    // LDS (wave_n vertices of 20 B: minima first, then labels, parents, ids).
    const int64_t ntiny = (int64_t)A.q->ntiny;
    if (ntiny == 0 || A.wave_n <= 0) return;
    const int wave = threadIdx.x / kWave;
    const int64_t wcap = A.wave_n;
    uint64_t* wbest = reinterpret_cast<uint64_t*>(reinterpret_cast<char*>(lds) +
                                                  (size_t)wave * (size_t)wcap * 20);
    int32_t* wlab = reinterpret_cast<int32_t*>(wbest + wcap);
    while (true) {
        uint32_t gi = 0;
        if (lane_id() == 0) gi = atomicAdd(&A.q->tiny_next, 1u);
        gi = __shfl(gi, 0, kWave);
        if ((int64_t)gi >= ntiny) break;
        solve_graph_wave(A, A.tiny[gi], wcap, wlab, wbest, wlab + wcap, wlab + 2 * wcap);
    }
}

// Clears the counters and the cooperative blocks, splits the order into the
// cooperative and other lists (stable), marks the batch start.  One workgroup.
constexpr int kPrepThreads = 1024;
__global__ __launch_bounds__(kPrepThreads) void k_batch_prep(BatchArgs A) {
    __shared__ uint32_t s_wave[kPrepThreads / kWave];
    if (threadIdx.x < sizeof(BatchQueue) / 4) reinterpret_cast<uint32_t*>(A.q)[threadIdx.x] = 0;
    uint32_t* xw = reinterpret_cast<uint32_t*>(A.xw);
    for (uint32_t i = threadIdx.x; i < kMaxXcd * sizeof(XcdWork) / 4; i += blockDim.x) xw[i] = 0;
    __syncthreads();
    if (threadIdx.x < kMaxXcd) A.xw[threadIdx.x].ticket = (uint64_t)kNotReady << 32;
    if (threadIdx.x == 0 && A.ticks) A.ticks[A.G] = kKeyMax;
    uint32_t nb = 0, ns = 0, nt = 0;
    for (int64_t base = 0; base < A.G; base += kPrepThreads) {
        const int64_t i = base + threadIdx.x;
        int64_t g = -1;
        bool big = false, tiny = false;
        if (i < A.G) {
            g = A.order ? (int64_t)A.order[i] : i;
            const int64_t m = A.eoff[g + 1] - A.eoff[g], n = A.voff[g + 1] - A.voff[g];
            big = A.coop_edges >= 0 && m >= A.coop_edges;
            tiny = !big && A.wave_n > 0 && m <= A.wave_edges && n >= 0 && n <= A.wave_n;
        }
        uint32_t tb, ts, tt;
        const uint32_t rb = block_rank<kPrepThreads>(big, s_wave, &tb);
        const uint32_t rs = block_rank<kPrepThreads>(i < A.G && !big && !tiny, s_wave, &ts);
        const uint32_t rt = block_rank<kPrepThreads>(tiny, s_wave, &tt);
        if (i < A.G) {
            if (big) A.big[nb + rb] = (int32_t)g;
            else if (tiny) A.tiny[nt + rt] = (int32_t)g;
            else A.small[ns + rs] = (int32_t)g;
        }
        nb += tb;
        ns += ts;
        nt += tt;
    }
    if (threadIdx.x == 0) {
        A.q->nbig = nb;
        A.q->nsmall = ns;
        A.q->ntiny = nt;
    }
}

size_t batch_slot_bytes(int64_t nmax) {
    const size_t cap = (size_t)(nmax > 0 ? nmax : 1);
    const size_t chunks = cap / ((size_t)kMinBatchBlock * kCoopVertsPerThread) + 2;
    return (cap * 20 + chunks * 4 + 255) / 256 * 256;
}

size_t batch_xslot_bytes(int64_t nmax) {
    return batch_slot_bytes(nmax) +
           ((size_t)kPairMax * (kPairMax - 1) / 2 * 8 + (size_t)kPairMax * 4 + 255) / 256 * 256;
}

BatchLayout batch_layout(int64_t G, int64_t nmax, int workgroups) {
    BatchLayout L;
    size_t off = (sizeof(BatchQueue) + 255) / 256 * 256;
    L.xw_off = off;
    off += (size_t)kMaxXcd * sizeof(XcdWork);
    L.lists_off = off;
    off += ((size_t)(G > 0 ? G : 1) * 12 + 255) / 256 * 256;
    L.xslots_off = off;
    off += (size_t)kMaxXcd * batch_xslot_bytes(nmax);
    L.wslots_off = off;
    off += (size_t)(workgroups > 0 ? workgroups : 1) * batch_slot_bytes(nmax);
    L.total = off;
    return L;
}

int launch_batch(const BatchArgs& A, int block, int workgroups, hipStream_t s) {
    const size_t lds = (size_t)A.lds_n * 20;
    hipLaunchKernelGGL(k_batch_prep, dim3(1), dim3(kPrepThreads), 0, s, A);
    switch (block) {
        case 256: hipLaunchKernelGGL(k_batch<256>, dim3(workgroups), dim3(256), lds, s, A); break;
        case 512: hipLaunchKernelGGL(k_batch<512>, dim3(workgroups), dim3(512), lds, s, A); break;
        default: hipLaunchKernelGGL(k_batch<1024>, dim3(workgroups), dim3(1024), lds, s, A); break;
    }
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

bool batch_allow_lds(int block, size_t bytes) {
    if (bytes <= 64 * 1024) return true;
    hipError_t e;
    switch (block) {
        case 256: e = hipFuncSetAttribute((const void*)k_batch<256>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes); break;
        case 512: e = hipFuncSetAttribute((const void*)k_batch<512>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes); break;
        default: e = hipFuncSetAttribute((const void*)k_batch<1024>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes); break;
    }
    if (e != hipSuccess) (void)hipGetLastError();
    return e == hipSuccess;
}

int batch_resident_workgroups(int block, size_t lds_bytes) {
    int per_cu = 0, dev = 0, cus = 0;
    hipError_t e;
    switch (block) {
        case 256: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch<256>, 256, lds_bytes); break;
        case 512: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch<512>, 512, lds_bytes); break;
        default: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch<1024>, 1024, lds_bytes); break;
    }
    if (e != hipSuccess || hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return per_cu * cus;
}

}  // namespace msf
