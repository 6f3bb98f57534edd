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

// Slot of the unordered pair {x, y}, x < y, in a triangular table.
__device__ __forceinline__ void slot_pair(int64_t s, int32_t& x, int32_t& y) {
    // y = largest integer with y (y - 1) / 2 <= s
    int64_t yy = (int64_t)((1.0 + sqrt(1.0 + 8.0 * (double)s)) * 0.5);
    while (yy * (yy - 1) / 2 > s) --yy;
    while ((yy + 1) * yy / 2 <= s) ++yy;
    y = (int32_t)yy;
    x = (int32_t)(s - yy * (yy - 1) / 2);
}

__global__ __launch_bounds__(kTailThreads) void k_tail(
    const uint64_t* __restrict__ pairs, int64_t nn, uint32_t* __restrict__ list_xy,
    uint64_t* __restrict__ list_key, const uint32_t* __restrict__ view_id,
    uint8_t* __restrict__ mask, const int32_t* __restrict__ orig_in, int32_t* __restrict__ rep,
    Ctrl* ctrl) {
    __shared__ uint64_t best[kTailMax];
    __shared__ int32_t comp[kTailMax];   // representative of each tail vertex's component
    __shared__ int32_t arg[kTailMax];    // list index of best[]
    __shared__ int32_t par[kTailMax];
    __shared__ uint32_t s_cnt, s_live, s_found, s_scan;
    const int tid = threadIdx.x;
    const int64_t nslots = nn * (nn - 1) / 2;
    if (tid == 0) s_cnt = 0;
    for (int v = tid; v < nn; v += blockDim.x) comp[v] = v;
    __syncthreads();
    for (int64_t s = tid; s < nslots; s += blockDim.x) {
        const uint64_t k = pairs[s];
        if (k == kKeyMax) continue;
        int32_t x, y;
        slot_pair(s, x, y);
        const uint32_t i = atomicAdd(&s_cnt, 1u);
        list_xy[i] = (uint32_t)x | ((uint32_t)y << 16);
        list_key[i] = k;
    }
    __syncthreads();
    const uint32_t L = s_cnt;
    uint64_t wsum = 0, nfound = 0;
    int round = 0;
    for (; round < kTailRoundsMax; ++round) {
        for (int v = tid; v < nn; v += blockDim.x) best[v] = kKeyMax;
        if (tid == 0) { s_live = 0; s_found = 0; s_scan = 0; }
        __syncthreads();
        uint32_t scanned = 0;
        for (uint32_t i = tid; i < L; i += blockDim.x) {          // lightest edges
            const uint32_t xy = list_xy[i];
            const int32_t x = comp[xy & 0xffff], y = comp[xy >> 16];
            if (x == y) continue;
            ++scanned;
            const uint64_t k = list_key[i];
            atomic_min_key(&best[x], k);
            atomic_min_key(&best[y], k);
        }
        if (scanned) atomicAdd(&s_scan, scanned);
        __syncthreads();
        for (uint32_t i = tid; i < L; i += blockDim.x) {          // which entry won
            const uint32_t xy = list_xy[i];
            const int32_t x = comp[xy & 0xffff], y = comp[xy >> 16];
            if (x == y) continue;
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
            const int32_t x = comp[xy & 0xffff], y = comp[xy >> 16];
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
            ctrl->tail_scan[round] = s_scan;
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
        for (int v = tid; v < nn; v += blockDim.x) comp[v] = par[comp[v]];
        __syncthreads();
    }
    wsum = wave_sum_u64(wsum);
    nfound = wave_sum_u64(nfound);
    if (lane_id() == 0 && nfound) {
        atomicAdd((unsigned long long*)&ctrl->total, (unsigned long long)wsum);
        atomicAdd((unsigned long long*)&ctrl->msf_edges, (unsigned long long)nfound);
    }
    if (tid == 0) {
        ctrl->tail_rounds = (uint32_t)round;
        ctrl->tail_edges = L;
        if (round == kTailRoundsMax) atomicOr(&ctrl->err, kErrInternal);
    }
}

void launch_tail(const uint64_t* pairs, int64_t nn, uint32_t* list_xy, uint64_t* list_key,
                 const uint32_t* view_id, uint8_t* mask, const int32_t* orig_in, int32_t* rep,
                 Ctrl* ctrl, hipStream_t s) {
    hipLaunchKernelGGL(k_tail, dim3(1), dim3(kTailThreads), 0, s, pairs, nn, list_xy, list_key,
                       view_id, mask, orig_in, rep, ctrl);
}

}  // namespace msf
