// Single-workgroup tail of the Borůvka loop (the paper's base case, Sec.
// IV-D, adapted: once few vertices are left, finish everything in one place).
//
// Input: the lightest edge of every pair of the <= kTailMax remaining
// vertices, produced by the last streaming pass (parallel edges already
// reduced to the lightest, which the paper allows in a round, Sec. II-C).
// Keys stay (w << 32 | position in the last edge layout), so the tie break is
// unchanged and the MSF edge id is recovered from the position.  All rounds
// run in LDS with workgroup barriers: no host round trips.
#include "prim.h"

namespace msf {

// Component pairs of the in-LDS dedup (64 KiB of keys: up to 128 components).
constexpr uint32_t kTailPairSlots = 8192;

__global__ __launch_bounds__(kTailThreads) void k_tail(
    const uint64_t* __restrict__ pairs, int64_t nn, uint32_t* list_xy0, uint64_t* list_key0,
    uint32_t* list_xy1, uint64_t* list_key1, const uint32_t* __restrict__ view_id,
    uint8_t* __restrict__ mask, const int32_t* __restrict__ orig_in, int32_t* __restrict__ rep,
    Ctrl* ctrl) {
    uint32_t* list_xy = list_xy0;
    uint64_t* list_key = list_key0;
    // The list always holds pairs of current component roots: it is rebuilt
    // after every round with both ends mapped through the hook forest, and
    // pairs that fell inside one component are dropped.
    __shared__ uint64_t best[kTailMax];
    __shared__ int32_t arg[kTailMax];    // list index of best[]
    __shared__ int32_t par[kTailMax];
    __shared__ uint32_t s_cnt, s_live, s_found;
    __shared__ uint64_t s_scan[kTailThreads / kWave];
    __shared__ int16_t s_dense[kTailMax];        // next-round component id of a root
    __shared__ int16_t s_inv[kTailMax];          // root of a next-round component id
    __shared__ unsigned long long s_pairs[kTailPairSlots];   // lightest entry per component pair
    const int tid = threadIdx.x;
    if (tid == 0) s_cnt = 0;
    __syncthreads();
    // List of the occupied slots: wave w walks rows y = w, w + 16, ... of the
    // triangle (slots y(y-1)/2 + x, x < y), 64 columns at a time, and appends
    // with one LDS atomic per step of the wave.
    {
        const int wave = tid / kWave, lane = tid % kWave;
        for (int64_t y = 1 + wave; y < nn; y += kTailThreads / kWave) {
            const int64_t row = y * (y - 1) / 2;
            for (int64_t x0 = 0; x0 < y; x0 += kWave) {
                const int64_t x = x0 + lane;
                const uint64_t k = x < y ? pairs[row + x] : kKeyMax;
                const uint64_t occ = __ballot(k != kKeyMax);
                if (occ == 0) continue;
                uint32_t base = 0;
                if (lane == 0) base = atomicAdd(&s_cnt, (uint32_t)__popcll(occ));
                base = __shfl(base, 0, kWave);
                if (k != kKeyMax) {
                    const uint32_t i = base + lanes_below(occ);
                    list_xy[i] = (uint32_t)x | ((uint32_t)y << 16);
                    list_key[i] = k;
                }
            }
        }
    }
    __syncthreads();
    uint32_t L = s_cnt;
    const uint32_t L0 = L;
    uint64_t wsum = 0, nfound = 0;
    int round = 0;
    for (; round < kTailRoundsMax; ++round) {
        for (int v = tid; v < nn; v += blockDim.x) best[v] = kKeyMax;
        if (tid == 0) { s_live = 0; s_found = 0; }
        __syncthreads();
        for (uint32_t i = tid; i < L; i += blockDim.x) {          // lightest edges
            const uint32_t xy = list_xy[i];
            const int32_t x = xy & 0xffff, y = xy >> 16;
            const uint64_t k = list_key[i];
            atomic_min_key(&best[x], k);
            atomic_min_key(&best[y], k);
        }
        __syncthreads();
        for (uint32_t i = tid; i < L; i += blockDim.x) {          // which entry won
            const uint32_t xy = list_xy[i];
            const int32_t x = xy & 0xffff, y = xy >> 16;
            const uint64_t k = list_key[i];
            if (best[x] == k) arg[x] = (int32_t)i;
            if (best[y] == k) arg[y] = (int32_t)i;
        }
        __syncthreads();
        uint32_t live = 0, found = 0;
        for (int v = tid; v < nn; v += blockDim.x) {              // hook + mark
            const uint64_t b = best[v];
            if (b == kKeyMax) { par[v] = v; continue; }
            ++live;
            const uint32_t xy = list_xy[arg[v]];
            const int32_t x = xy & 0xffff, y = xy >> 16;
            const int32_t other = x == v ? y : x;
            if (best[other] == b && v < other) {
                par[v] = v;
            } else {
                par[v] = other;
                const uint32_t pos = (uint32_t)b;
                mask[view_id ? view_id[pos] : pos] = 1;
                wsum += b >> 32;
                ++found;
            }
        }
        if (live) atomicAdd(&s_live, live);
        if (found) atomicAdd(&s_found, found);
        __syncthreads();
        if (s_live == 0) break;
        if (tid == 0) {
            ctrl->tail_live[round] = s_live;
            ctrl->tail_found[round] = s_found;
            ctrl->tail_scan[round] = L;
        }
        nfound += found;
        for (int it = 0; it < 11; ++it) {                         // pointer doubling
            int32_t g[kTailMax / kTailThreads];
            int c = 0;
            for (int v = tid; v < nn; v += blockDim.x) g[c++] = par[par[v]];
            __syncthreads();
            c = 0;
            for (int v = tid; v < nn; v += blockDim.x) par[v] = g[c++];
            __syncthreads();
        }
        if (rep) {
            for (int v = tid; v < nn; v += blockDim.x) {
                if (best[v] != kKeyMax && par[v] != v)
                    rep[orig_in ? orig_in[v] : v] = orig_in ? orig_in[par[v]] : par[v];
            }
        }
        if (tid == 0) s_cnt = 0;
        // Dense ids of the next round's components (roots that have an edge).
        const bool root = tid < nn && par[tid] == tid && best[tid] != kKeyMax;
        uint64_t nd64;
        const uint32_t d = (uint32_t)block_excl_scan(root ? 1 : 0, s_scan, &nd64);
        const uint32_t nd = (uint32_t)nd64;
        if (root) { s_dense[tid] = (int16_t)d; s_inv[d] = (int16_t)tid; }
        const bool dedup = nd >= 2 && (uint64_t)nd * (nd - 1) / 2 <= kTailPairSlots;
        if (dedup)
            for (uint32_t i = tid; i < nd * (nd - 1) / 2; i += kTailThreads) s_pairs[i] = kKeyMax;
        __syncthreads();
        if (dedup) {
            // Few components left: keep only the lightest entry per component
            // pair (parallel edges are dropped, as the paper allows).
            for (uint32_t i = tid; i < L; i += kTailThreads) {
                const uint32_t xy = list_xy[i];
                const int32_t x = par[xy & 0xffff], y = par[xy >> 16];
                if (x == y) continue;
                const uint32_t dx = (uint32_t)s_dense[x], dy = (uint32_t)s_dense[y];
                const uint32_t lo = dx < dy ? dx : dy, hi = dx < dy ? dy : dx;
                const uint64_t k = list_key[i];
                unsigned long long* slot = &s_pairs[(hi * (hi - 1) / 2 + lo) & (kTailPairSlots - 1)];
                if (k < *slot) atomicMin(slot, (unsigned long long)k);
            }
            __syncthreads();
            uint32_t* xy_out = list_xy == list_xy0 ? list_xy1 : list_xy0;
            uint64_t* key_out = list_key == list_key0 ? list_key1 : list_key0;
            const int wave = tid / kWave, lane = tid % kWave;
            for (uint32_t y = 1 + wave; y < nd; y += kTailThreads / kWave) {
                const uint32_t row = y * (y - 1) / 2;
                for (uint32_t x0 = 0; x0 < y; x0 += kWave) {
                    const uint32_t x = x0 + lane;
                    const uint64_t k = x < y ? s_pairs[row + x] : kKeyMax;
                    const uint64_t occ = __ballot(k != kKeyMax);
                    if (occ == 0) continue;
                    uint32_t base = 0;
                    if (lane == 0) base = atomicAdd(&s_cnt, (uint32_t)__popcll(occ));
                    base = __shfl(base, 0, kWave);
                    if (k != kKeyMax) {
                        const uint32_t j = base + lanes_below(occ);
                        xy_out[j] = (uint32_t)(uint16_t)s_inv[x] | ((uint32_t)(uint16_t)s_inv[y] << 16);
                        key_out[j] = k;
                    }
                }
            }
            list_xy = xy_out;
            list_key = key_out;
        } else {
            // Next round's list, in the other buffer: both ends mapped to
            // their new roots, pairs inside one component dropped.
            uint32_t* xy_out = list_xy == list_xy0 ? list_xy1 : list_xy0;
            uint64_t* key_out = list_key == list_key0 ? list_key1 : list_key0;
            const int wave = tid / kWave, lane = tid % kWave;
            for (uint32_t i0 = (uint32_t)wave * kWave; i0 < L; i0 += kTailThreads) {
                const uint32_t i = i0 + lane;
                int32_t x = 0, y = 0;
                if (i < L) {
                    const uint32_t xy = list_xy[i];
                    x = par[xy & 0xffff];
                    y = par[xy >> 16];
                }
                const uint64_t live = __ballot(i < L && x != y);
                if (live == 0) continue;
                uint32_t base = 0;
                if (lane == 0) base = atomicAdd(&s_cnt, (uint32_t)__popcll(live));
                base = __shfl(base, 0, kWave);
                if ((live >> lane) & 1) {
                    const uint32_t j = base + lanes_below(live);
                    xy_out[j] = (uint32_t)x | ((uint32_t)y << 16);
                    key_out[j] = list_key[i];
                }
            }
            list_xy = xy_out;
            list_key = key_out;
        }
        __syncthreads();
        L = s_cnt;
    }
    wsum = wave_sum_u64(wsum);
    nfound = wave_sum_u64(nfound);
    if (lane_id() == 0 && nfound) {
        atomicAdd((unsigned long long*)&ctrl->total, (unsigned long long)wsum);
        atomicAdd((unsigned long long*)&ctrl->msf_edges, (unsigned long long)nfound);
    }
    if (tid == 0) {
        ctrl->tail_rounds = (uint32_t)round;
        ctrl->tail_edges = L0;
        if (round == kTailRoundsMax) atomicOr(&ctrl->err, kErrInternal);
    }
}

void launch_tail(const uint64_t* pairs, int64_t nn, uint32_t* const list_xy[2],
                 uint64_t* const list_key[2], const uint32_t* view_id, uint8_t* mask,
                 const int32_t* orig_in, int32_t* rep, Ctrl* ctrl, hipStream_t s) {
    hipLaunchKernelGGL(k_tail, dim3(1), dim3(kTailThreads), 0, s, pairs, nn, list_xy[0],
                       list_key[0], list_xy[1], list_key[1], view_id, mask, orig_in, rep, ctrl);
}

}  // namespace msf
