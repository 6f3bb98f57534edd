// Batched MSF: thousands of independent graphs in one persistent launch.
//
// Each workgroup repeatedly takes the next graph from an atomic work queue
// (the caller may pass an order, e.g. largest first) and runs every Borůvka
// round of that graph itself (paper Sec. II-C): lightest incident edge per
// vertex with packed (w << 32 | local edge index) keys, hook with the 2-cycle
// tie break and MSF marking, pointer jumping, dense relabelling of the roots,
// composition of the labels of the graph's vertices.  Phases are separated by
// workgroup barriers only, so the whole batch needs no host round trip and the
// launch can be captured in a hipGraph.  A graph's per-vertex state (label,
// best key, parent, new id: 20 B per vertex) lives in LDS when the graph is
// small enough, else in a global scratch slot owned by the workgroup.
#include "batch.h"
#include "prim.h"

namespace msf {

constexpr int kBatchMaxRounds = 64;
constexpr int kEdgeIlp = 4;

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
__device__ void solve_graph(const BatchArgs& A, int64_t g, int32_t* lab, uint64_t* best,
                            int32_t* par, int32_t* nid, uint32_t* s_wave) {
    const int tid = threadIdx.x;
    const int64_t e0 = A.eoff[g];
    const int64_t m = A.eoff[g + 1] - e0;
    const int64_t n = A.voff[g + 1] - A.voff[g];
    const int32_t* U = A.u + e0;
    const int32_t* V = A.v + e0;
    const uint32_t* W = A.w + e0;
    uint8_t* mask = A.mask + e0;
    const bool bad_shape = n < 0 || n > A.nmax || m < 0 || m > 0xffffffffLL;
    bool bad = bad_shape;
    uint64_t wsum = 0;
    if (!bad_shape) {
        for (int64_t i = tid; i < m; i += BS) mask[i] = 0;
        for (int64_t x = tid; x < n; x += BS) lab[x] = (int32_t)x;
        int64_t ncur = n;
        __syncthreads();
        for (int round = 0; round < kBatchMaxRounds && ncur > 1; ++round) {
            for (int64_t x = tid; x < ncur; x += BS) best[x] = kKeyMax;
            __syncthreads();
            int any = 0;
            // lightest edges, kEdgeIlp independent edges per thread: all loads
            // and label gathers of a step are issued before any is used
            for (int64_t base = 0; base < m; base += (int64_t)BS * kEdgeIlp) {
                int32_t a[kEdgeIlp], b[kEdgeIlp], la[kEdgeIlp], lb[kEdgeIlp];
                uint32_t wt[kEdgeIlp];
#pragma unroll
                for (int k = 0; k < kEdgeIlp; ++k) {
                    const int64_t e = base + k * BS + tid;
                    a[k] = b[k] = 0;
                    wt[k] = 0;
                    if (e < m) { a[k] = U[e]; b[k] = V[e]; wt[k] = W[e]; }
                }
#pragma unroll
                for (int k = 0; k < kEdgeIlp; ++k) {
                    const int64_t e = base + k * BS + tid;
                    la[k] = lb[k] = -1;                       // dead unless set below
                    if (e >= m || a[k] == b[k]) continue;
                    if (round == 0) {                         // labels are the ids
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
#pragma unroll
                for (int k = 0; k < kEdgeIlp; ++k) {
                    if (la[k] == lb[k]) continue;
                    const int64_t e = base + k * BS + tid;
                    any = 1;
                    const uint64_t key = ((uint64_t)wt[k] << 32) | (uint64_t)e;
                    atomic_min_key(&best[la[k]], key);
                    atomic_min_key(&best[lb[k]], key);
                }
            }
            if (!__syncthreads_or(any) || __syncthreads_or(bad)) break;
            for (int64_t x = tid; x < ncur; x += BS) {                // hook + mark
                const uint64_t b = best[x];
                if (b == kKeyMax) { par[x] = (int32_t)x; continue; }
                const uint32_t pos = (uint32_t)b;
                const int32_t la = lab[U[pos]], lb = lab[V[pos]];
                const int32_t other = la == (int32_t)x ? lb : la;
                if (best[other] == b && (int32_t)x < other) {
                    par[x] = (int32_t)x;
                } else {
                    par[x] = other;
                    mask[pos] = 1;
                    wsum += b >> 32;
                }
            }
            __syncthreads();
            for (int it = 0; it < 64; ++it) {                          // pointer jumping
                int changed = 0;
                for (int64_t x = tid; x < ncur; x += BS) {
                    const int32_t p = par[x], pp = par[p];
                    if (p != pp) { par[x] = pp; changed = 1; }
                }
                if (!__syncthreads_or(changed)) break;
            }
            int64_t roots = 0;                                         // dense ids of roots
            for (int64_t base = 0; base < ncur; base += BS) {
                const int64_t x = base + tid;
                const bool r = x < ncur && par[x] == (int32_t)x && best[x] != kKeyMax;
                uint32_t tot;
                const uint32_t rk = block_rank<BS>(r, s_wave, &tot);
                if (r) nid[x] = (int32_t)(roots + rk);
                roots += tot;
            }
            __syncthreads();
            for (int64_t i = tid; i < n; i += BS) {                    // compose labels
                const int32_t l = lab[i];
                if (l >= 0) lab[i] = best[l] == kKeyMax ? -1 : nid[par[l]];
            }
            ncur = roots;
            __syncthreads();
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

template <int BS>
__global__ __launch_bounds__(BS) void k_batch(BatchArgs A) {
    extern __shared__ uint64_t lds[];
    __shared__ uint32_t s_wave[BS / kWave];
    __shared__ int64_t s_g;
    if (threadIdx.x == 0 && A.ticks) atomicMin((unsigned long long*)&A.ticks[A.G],
                                               (unsigned long long)wall_clock64());
    char* slot = A.scratch + (size_t)blockIdx.x * A.slot_bytes;
    while (true) {
        if (threadIdx.x == 0) s_g = (int64_t)atomicAdd(A.queue, 1u);
        __syncthreads();
        const int64_t gi = s_g;
        __syncthreads();
        if (gi >= A.G) break;
        const int64_t g = A.order ? (int64_t)A.order[gi] : gi;
        const int64_t n = A.voff[g + 1] - A.voff[g];
        if (n <= A.lds_n) {
            const int64_t cap = A.lds_n;
            uint64_t* best = lds;
            int32_t* lab = reinterpret_cast<int32_t*>(lds + cap);
            int32_t* par = lab + cap;
            int32_t* nid = par + cap;
            solve_graph<BS>(A, g, lab, best, par, nid, s_wave);
        } else {
            const size_t cap = (size_t)A.nmax;
            uint64_t* best = reinterpret_cast<uint64_t*>(slot);
            int32_t* lab = reinterpret_cast<int32_t*>(slot + cap * 8);
            int32_t* par = lab + cap;
            int32_t* nid = par + cap;
            solve_graph<BS>(A, g, lab, best, par, nid, s_wave);
        }
    }
}

__global__ void k_batch_prep(uint32_t* queue, uint64_t* ticks, int64_t G) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        *queue = 0;
        if (ticks) ticks[G] = kKeyMax;
    }
}

size_t batch_slot_bytes(int64_t nmax) {
    return ((size_t)(nmax > 0 ? nmax : 1) * 20 + 255) / 256 * 256;
}

// Launches the batch; `workgroups` slots of slot_bytes each must follow `scratch`.
int launch_batch(const BatchArgs& A0, int block, int workgroups, hipStream_t s) {
    BatchArgs A = A0;
    A.slot_bytes = batch_slot_bytes(A.nmax);
    const size_t lds = (size_t)A.lds_n * 20;
    hipLaunchKernelGGL(k_batch_prep, dim3(1), dim3(64), 0, s, A.queue, A.ticks, A.G);
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

}  // namespace msf
