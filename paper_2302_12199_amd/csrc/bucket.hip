// Round 0 of Borůvka by vertex buckets (paper Sec. II-C: the lightest
// incident edge of every vertex, then the relabelling of every edge).
//
// Done directly on the caller's edge list, both steps touch an n-sized table
// at two random places per edge.  With no locality in the vertex ids (RMAT
// with permuted ids) every touch is a separate 128-byte line request to HBM,
// and the min updates are device-scope atomics that do not stay in the XCD's
// L2.  Here every random access goes to LDS instead, and global memory is
// only streamed or read in runs:
//
//   scatter  per tile of 2^13 edges: the tile's arcs (one per endpoint) are
//            sorted by vertex bucket (2^14 vertices) in LDS and written as one
//            contiguous block; meta[t][b] = (run start, length)
//   index    meta transposed to bucket-major; bucket totals; their scan
//   min      one workgroup per bucket: its runs (one per tile) are read 1024
//            runs at a time, each arc's lane found by a branchless search over
//            the batch's run prefix; the minimum key per vertex is kept in LDS.
//            It also writes the arcs' vertex indices as one bucket-major
//            stream and where each run starts in it
//   hot      (after hook / jump / root scan) the round-1 labels renumbered by
//            how often sampled edge ends carry them, most frequent first
//   label    one workgroup per bucket: the bucket's labels in LDS, the index
//            stream in, the labels out
//   pass     per tile: its runs of labels are gathered into LDS in
//            tile-block order; each edge reads its two labels there (found by
//            its arc places; the endpoints are not read again), and the pass
//            writes the relabelled layout and runs the next round's
//            lightest-edge search, the minima of the first labels in LDS
#include <algorithm>

#include "bucket.h"
#include "host.h"
#include "launch.h"
#include "prim.h"

namespace msf {

size_t scan_levels_bytes(int64_t n);
void launch_scan_u64(uint64_t* cnt, int64_t n, uint64_t* tmp, uint64_t* total, hipStream_t s);

namespace {

constexpr size_t kAl = 256;
size_t al(size_t x) { return (x + kAl - 1) / kAl * kAl; }
int64_t nbuckets(int64_t n) { return (n + kBucketWidth - 1) >> kBucketShift; }
int64_t ntiles(int64_t m) { return (m + kBucketTile - 1) >> kBucketTileShift; }
constexpr int kGroups = (int)(kBucketTile / 4 / kBucketThreads);   // 4-edge groups per thread
constexpr uint32_t kArcMask = (uint32_t)kTileArcs - 1;
constexpr int kInFlight = 16;                                       // gathers per lane in flight
constexpr int kHotSample = 65535;                                   // edge ends sampled for hot labels
constexpr uint32_t kHotIds = 10240;                                 // labels whose minima stay in LDS
constexpr uint32_t kPassGrid = 256;   // workgroups of the pass: one per CU, tiles taken grid-stride
constexpr uint32_t kScatterGrid = 1024;                             // workgroups of the scatter
constexpr int kPassThreads = 1024;    // one pass workgroup per CU (LDS)
constexpr int kPassParts = (int)(kBucketTile / 4 / kPassThreads / kGroups);   // edge parts per tile

template <typename T, typename V>
__device__ __forceinline__ void load4(const T* __restrict__ p, int64_t q, int64_t e1, T (&x)[4]) {
    const int64_t e = q * 4;
    if (e + 3 < e1) {
        const V t = reinterpret_cast<const V*>(p)[q];
        x[0] = t.x; x[1] = t.y; x[2] = t.z; x[3] = t.w;
    } else {
#pragma unroll
        for (int k = 0; k < 4; ++k) x[k] = e + k < e1 ? p[e + k] : 0;
    }
}

// As load4 for data read once: non-temporal loads, which leave the L2 to the
// tables that are read again.
__device__ __forceinline__ void load4_nt(const uint32_t* __restrict__ p, int64_t q, int64_t e1,
                                         uint32_t (&x)[4]) {
    const int64_t e = q * 4;
    typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
    if (e + 3 < e1) {
        const u32x4 t = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(p) + q);
        x[0] = t.x; x[1] = t.y; x[2] = t.z; x[3] = t.w;
    } else {
#pragma unroll
        for (int k = 0; k < 4; ++k) x[k] = e + k < e1 ? __builtin_nontemporal_load(p + e + k) : 0;
    }
}

__device__ __forceinline__ bool in_range(int32_t a, int32_t b, int64_t n) {
    return (uint32_t)a < (uint64_t)n && (uint32_t)b < (uint64_t)n;
}

// Largest k in [0, kBucketMax) with a[k] <= x (a non-decreasing, a[0] <= x): ten
// fixed steps, so a lane's searches interleave.  With empty runs (equal
// starts) it lands on the one run that holds slot x.
__device__ __forceinline__ uint32_t last_le(const uint32_t* a, uint32_t x) {
    uint32_t lo = 0;
#pragma unroll
    for (uint32_t step = kBucketMax / 2; step > 0; step >>= 1)
        lo = a[lo + step] <= x ? lo + step : lo;
    return lo;
}
static_assert(kBucketMax == kBucketThreads, "a batch of runs has one entry per thread");

}  // namespace

bool bucket_eligible(int64_t m, int64_t n) {
    return n >= (1ll << 21) && nbuckets(n) <= kBucketMax && m >= (1ll << 22) && m < (1ll << 31);
}

size_t bucket_carve(char* ws, int64_t m, int64_t n, BucketBuffers* B) {
    BucketBuffers b{};
    if (!bucket_eligible(m, n)) {
        if (B) *B = b;
        return 0;
    }
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += al(bytes);
        return ws ? ws + o : nullptr;
    };
    const int64_t nb = nbuckets(n), nt = ntiles(m), cells = nb * nt;
    b.arcs = (uint64_t*)take((size_t)(nt * kTileArcs) * 8);
    b.meta = (uint32_t*)take((size_t)cells * 4);
    b.metat = (uint32_t*)take((size_t)cells * 4);
    b.offb = (uint32_t*)take((size_t)cells * 4);
    b.offt = (uint32_t*)take((size_t)cells * 4);
    b.base = (uint64_t*)take((size_t)(nb + 1) * 8);
    b.tmp = (uint64_t*)take(scan_levels_bytes(nb));
    b.xs = (uint16_t*)take((size_t)(2 * m + 64) * 2);   // 8-index groups may read past the end
    b.rank = (uint32_t*)take((size_t)m * 4 + 16);
    b.hotpre = (uint64_t*)take((size_t)(n + 2) * 8);
    b.hottmp = (uint64_t*)take(scan_levels_bytes(n + 1));
    b.hotn = -1;
    b.mcap = m;
    b.ncap = n;
    if (B) *B = b;
    return off;
}

bool bucket_usable(const BucketBuffers& B, int64_t m, int64_t n) {
    return B.arcs && bucket_eligible(m, n) && m <= B.mcap && n <= B.ncap;
}

// ---------------------------------------------------------------- scatter

// Arc of endpoint x of edge e (in tile block order): w << 32 | (e - e0) << 14
// | x mod 2^14.  An edge whose ids are out of range raises kErrRange and, like a
// self-loop, has no arcs.  rank[e] = places of its two arcs in the block.
__device__ __forceinline__ void load_ends_of_tile(const int32_t* __restrict__ u,
                                                  const int32_t* __restrict__ v, int64_t m,
                                                  uint32_t t, int32_t (&a)[kGroups][4],
                                                  int32_t (&b)[kGroups][4]) {
    const int64_t e0 = (int64_t)t << kBucketTileShift;
    const int64_t e1 = e0 + kBucketTile < m ? e0 + kBucketTile : m;
#pragma unroll
    for (int j = 0; j < kGroups; ++j) {
        const int64_t q = e0 / 4 + threadIdx.x + (int64_t)j * blockDim.x;
        load4<int32_t, int4>(u, q, e1, a[j]);
        load4<int32_t, int4>(v, q, e1, b[j]);
    }
}

// Tiles are taken grid-stride; the next tile's endpoints are loaded while
// the current tile's arcs are placed and written, a tile's weights while its
// arcs are counted.
__global__ __launch_bounds__(kBucketThreads) void k_bk_scatter(
    const int32_t* __restrict__ u, const int32_t* __restrict__ v, const uint32_t* __restrict__ w,
    int64_t m, int64_t n, uint32_t nb, uint32_t nt, uint64_t* __restrict__ arcs,
    uint32_t* __restrict__ meta, uint32_t* __restrict__ rank, Ctrl* ctrl) {
    __shared__ __align__(16) uint64_t s_stage[kTileArcs];
    __shared__ uint32_t s_cnt[kBucketMax];
    __shared__ uint32_t s_cur[kBucketMax];
    __shared__ uint64_t s_w[kBucketThreads / kWave];
    const int tid = threadIdx.x;
    bool bad = false;
    int32_t a[kGroups][4], b[kGroups][4];
    if (blockIdx.x < nt) load_ends_of_tile(u, v, m, blockIdx.x, a, b);
    for (uint32_t t = blockIdx.x; t < nt; t += gridDim.x) {
        const int64_t e0 = (int64_t)t << kBucketTileShift;
        const int64_t e1 = e0 + kBucketTile < m ? e0 + kBucketTile : m;
        uint32_t ww[kGroups][4];
#pragma unroll
        for (int j = 0; j < kGroups; ++j)
            load4<uint32_t, uint4>(w, e0 / 4 + tid + (int64_t)j * blockDim.x, e1, ww[j]);
        if (tid < (int)nb) s_cnt[tid] = 0;
        __syncthreads();
#pragma unroll
        for (int j = 0; j < kGroups; ++j) {
            const int64_t q = e0 / 4 + tid + (int64_t)j * blockDim.x;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                if (q * 4 + k >= e1) continue;
                const int32_t x = a[j][k], y = b[j][k];
                if (!in_range(x, y, n)) { bad = true; continue; }
                if (x == y) continue;
                atomicAdd(&s_cnt[(uint32_t)x >> kBucketShift], 1u);
                atomicAdd(&s_cnt[(uint32_t)y >> kBucketShift], 1u);
            }
        }
        __syncthreads();
        const uint32_t c = tid < (int)nb ? s_cnt[tid] : 0u;
        uint64_t tot;
        const uint32_t ex = (uint32_t)block_excl_scan(c, s_w, &tot);
        if (tid < (int)nb) {
            s_cur[tid] = ex;
            meta[(int64_t)t * nb + tid] = ex | (c << 16);
        }
        __syncthreads();
        int32_t a2[kGroups][4], b2[kGroups][4];
        const uint32_t tn = t + gridDim.x;
        if (tn < nt) load_ends_of_tile(u, v, m, tn, a2, b2);
#pragma unroll
        for (int j = 0; j < kGroups; ++j) {
            const int64_t q = e0 / 4 + tid + (int64_t)j * blockDim.x;
            uint32_t rk[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                rk[k] = 0;
                const int64_t e = q * 4 + k;
                const int32_t x = a[j][k], y = b[j][k];
                if (e >= e1 || !in_range(x, y, n) || x == y) continue;
                const uint64_t hi = ((uint64_t)ww[j][k] << 32) | ((uint64_t)(e - e0) << kBucketShift);
                const uint32_t px = atomicAdd(&s_cur[(uint32_t)x >> kBucketShift], 1u) & kArcMask;
                const uint32_t py = atomicAdd(&s_cur[(uint32_t)y >> kBucketShift], 1u) & kArcMask;
                s_stage[px] = hi | (uint64_t)(x & (kBucketWidth - 1));
                s_stage[py] = hi | (1ull << kArcSideBit) | (uint64_t)(y & (kBucketWidth - 1));
                rk[k] = px | (py << 16);
            }
            if (q * 4 + 3 < e1) {
                reinterpret_cast<uint4*>(rank)[q] = make_uint4(rk[0], rk[1], rk[2], rk[3]);
            } else {
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    if (q * 4 + k < e1) rank[q * 4 + k] = rk[k];
            }
        }
        __syncthreads();
        const uint32_t na = (uint32_t)(tot < (uint64_t)kTileArcs ? tot : (uint64_t)kTileArcs);
        uint64_t* dst = arcs + (int64_t)t * kTileArcs;   // 16-byte aligned (kTileArcs even)
        for (uint32_t i = tid; i < na / 2; i += blockDim.x)
            reinterpret_cast<uint4*>(dst)[i] = reinterpret_cast<const uint4*>(s_stage)[i];
        if ((na & 1) && tid == 0) dst[na - 1] = s_stage[na - 1];
        if (tn < nt) {
#pragma unroll
            for (int j = 0; j < kGroups; ++j)
#pragma unroll
                for (int k = 0; k < 4; ++k) { a[j][k] = a2[j][k]; b[j][k] = b2[j][k]; }
        }
    }
    if (__ballot(bad) && lane_id() == 0) atomicOr(&ctrl->err, kErrRange);
}

// ------------------------------------------------------------------ index

// out[c * R + r] = in[r * C + c] for an R x C matrix, 32 x 32 tiles.
__global__ __launch_bounds__(256) void k_transpose_u32(const uint32_t* __restrict__ in,
                                                       uint32_t* __restrict__ out, int64_t R,
                                                       int64_t C) {
    __shared__ uint32_t tile[32][33];
    const int64_t tiles_c = (C + 31) / 32;
    const int64_t tc = blockIdx.x % tiles_c, tr = blockIdx.x / tiles_c;
    const int tx = threadIdx.x % 32, ty = threadIdx.x / 32;
    for (int k = ty; k < 32; k += 8) {
        const int64_t r = tr * 32 + k, c = tc * 32 + tx;
        if (r < R && c < C) tile[k][tx] = in[r * C + c];
    }
    __syncthreads();
    for (int k = ty; k < 32; k += 8) {
        const int64_t c = tc * 32 + k, r = tr * 32 + tx;
        if (r < R && c < C) out[c * R + r] = tile[tx][k];
    }
}

// base[b] = arcs of bucket b (scanned afterwards).
__global__ __launch_bounds__(256) void k_bk_totals(const uint32_t* __restrict__ metat, uint32_t nt,
                                                   uint64_t* __restrict__ base) {
    __shared__ uint64_t s_w[256 / kWave];
    const uint32_t* row = metat + (int64_t)blockIdx.x * nt;
    uint64_t sum = 0;
    for (uint32_t t = threadIdx.x; t < nt; t += blockDim.x) sum += row[t] >> 16;
    uint64_t tot;
    (void)block_excl_scan(sum, s_w, &tot);
    if (threadIdx.x == 0) base[blockIdx.x] = tot;
}

// -------------------------------------------------------------------- min

__global__ __launch_bounds__(kBucketThreads) void k_bk_min(
    const uint64_t* __restrict__ arcs, const uint32_t* __restrict__ metat, uint32_t nt,
    int64_t n, int64_t narcs, const uint64_t* __restrict__ base, uint64_t* __restrict__ best,
    uint16_t* __restrict__ xs, uint32_t* __restrict__ offb) {
    __shared__ unsigned long long s_best[kBucketWidth];
    __shared__ uint32_t s_pre[kBucketThreads];   // batch run r0 + k starts at arc s_pre[k] of the batch
    __shared__ uint32_t s_rs[kBucketThreads];    // and at slot s_rs[k] of its tile block
    __shared__ uint64_t s_w[kBucketThreads / kWave];
    const uint32_t bk = xcd_slot(blockIdx.x, gridDim.x);   // neighbouring buckets on one XCD
    const int tid = threadIdx.x;
    for (int i = tid; i < kBucketWidth; i += blockDim.x) s_best[i] = kKeyMax;
    const uint64_t xs0 = base[bk];
    const uint32_t* row = metat + (int64_t)bk * nt;
    uint32_t pre = 0;   // arcs of the bucket in earlier batches
    uint32_t mt_next = (uint32_t)tid < nt ? row[tid] : 0u;
    for (uint32_t r0 = 0; r0 < nt; r0 += kBucketThreads) {
        const uint32_t r = r0 + tid;
        const uint32_t mt = mt_next;
        // the next batch's run entry, in flight while this batch's arcs load
        const uint32_t rn = r + kBucketThreads;
        mt_next = rn < nt ? row[rn] : 0u;
        uint64_t btot;
        const uint32_t ex = (uint32_t)block_excl_scan(mt >> 16, s_w, &btot);
        s_pre[tid] = ex;
        s_rs[tid] = mt & 0xffff;
        if (r < nt) offb[(int64_t)bk * nt + r] = pre + ex;
        __syncthreads();
        const uint32_t bt = (uint32_t)btot;
        for (uint32_t v0 = tid; v0 < bt; v0 += kInFlight * kBucketThreads) {
            uint64_t arc[kInFlight];
            uint32_t run[kInFlight];
#pragma unroll
            for (int k = 0; k < kInFlight; ++k) {
                const uint32_t x = v0 + k * kBucketThreads;
                arc[k] = 0;
                run[k] = 0;
                if (x < bt) {
                    const uint32_t j = last_le(s_pre, x);
                    run[k] = j;
                    const uint32_t slot = (s_rs[j] + (x - s_pre[j])) & kArcMask;
                    arc[k] = arcs[(int64_t)(r0 + j) * kTileArcs + slot];
                }
            }
#pragma unroll
            for (int k = 0; k < kInFlight; ++k) {
                const uint32_t x = v0 + k * kBucketThreads;
                if (x >= bt) continue;
                const uint32_t xl = (uint32_t)arc[k] & (uint32_t)(kBucketWidth - 1);
                const uint64_t e = ((uint64_t)(r0 + run[k]) << kBucketTileShift) +
                                   (((uint32_t)arc[k] >> kBucketShift) & (uint32_t)(kBucketTile - 1));
                const uint64_t key = (arc[k] & 0xffffffff00000000ull) | (e << 1) |
                                     (((uint32_t)arc[k] >> kArcSideBit) & 1u);
                if (key < s_best[xl]) atomicMin(&s_best[xl], (unsigned long long)key);
                const uint64_t o = xs0 + pre + x;
                if (o < (uint64_t)narcs) xs[o] = (uint16_t)xl;
            }
        }
        pre += bt;
        __syncthreads();
    }
    const int64_t v0 = (int64_t)bk << kBucketShift;
    for (int i = tid; i < kBucketWidth && v0 + i < n; i += blockDim.x) best[v0 + i] = s_best[i];
}

// ------------------------------------------------------------------ label

// relab[i] = M[vertex of arc i] over the bucket's part of the bucket-major
// streams, 8 indices (16 B) per group; relab shares memory with the arcs.
__global__ __launch_bounds__(kBucketThreads) void k_bk_label(
    const uint16_t* __restrict__ xs, const uint64_t* __restrict__ base, int64_t n, int64_t narcs,
    const int32_t* __restrict__ M, uint32_t* __restrict__ relab) {
    __shared__ uint32_t s_lab[kBucketWidth];
    const uint32_t bk = blockIdx.x;
    const int64_t v0 = (int64_t)bk << kBucketShift;
    for (int i = threadIdx.x; i < kBucketWidth; i += blockDim.x)
        s_lab[i] = v0 + i < n ? (uint32_t)M[v0 + i] : 0u;
    __syncthreads();
    const int64_t i1 = std::min((int64_t)base[bk + 1], narcs);
    const int64_t i0 = std::min((int64_t)base[bk], i1);
    const int64_t g0 = i0 / 8, g1 = (i1 + 7) / 8;
    const int64_t stride = blockDim.x;
    constexpr int kLabGroups = 8;   // 16-byte index groups per lane in flight
    for (int64_t gb = g0 + threadIdx.x; gb < g1; gb += kLabGroups * stride) {
        uint4 xv[kLabGroups];
#pragma unroll
        for (int j = 0; j < kLabGroups; ++j) {
            const int64_t g = gb + j * stride;
            if (g < g1) xv[j] = reinterpret_cast<const uint4*>(xs)[g];
        }
#pragma unroll
        for (int j = 0; j < kLabGroups; ++j) {
            const int64_t g = gb + j * stride;
            if (g >= g1) continue;
            const uint32_t wd[4] = {xv[j].x, xv[j].y, xv[j].z, xv[j].w};
            uint32_t r[8];
#pragma unroll
            for (int a = 0; a < 8; ++a)
                r[a] = s_lab[((a & 1) ? (wd[a >> 1] >> 16) : wd[a >> 1]) & (uint32_t)(kBucketWidth - 1)];
            const int64_t i = g * 8;
            if (i >= i0 && i + 8 <= i1) {
                reinterpret_cast<uint4*>(relab)[2 * g] = make_uint4(r[0], r[1], r[2], r[3]);
                reinterpret_cast<uint4*>(relab)[2 * g + 1] = make_uint4(r[4], r[5], r[6], r[7]);
            } else {
#pragma unroll
                for (int a = 0; a < 8; ++a)
                    if (i + a >= i0 && i + a < i1) relab[i + a] = r[a];
            }
        }
    }
}

// ------------------------------------------------------------------- pass

// Workgroups of 1024 threads take tiles grid-stride.  Slot x
// of a tile block holds the arc whose label is
// relab[base[b] + offt[t][b] + (x - run start of b)], b the bucket whose run
// holds x.  The labels are gathered into LDS in block order; an edge finds
// its two at the places recorded in rank[].  Then, as the plain relabelling
// pass does: dead edges (self-loops, equal labels) are written as (0, 0),
// live ones as label pairs, and take part in the next round's lightest-edge
// search with side keys (w << 32 | position << 1 | side, side 1 at the v end).
template <int OUT>
__global__ __launch_bounds__(kPassThreads) void k_bk_pass(
    const uint32_t* __restrict__ w, int64_t m, uint32_t nb, uint32_t nt,
    const uint32_t* __restrict__ meta,
    const uint32_t* __restrict__ offt, const uint64_t* __restrict__ base,
    const uint32_t* __restrict__ relab, const uint32_t* __restrict__ rank,
    int32_t* __restrict__ ou, int32_t* __restrict__ ov, uint32_t* __restrict__ op16,
    uint64_t* __restrict__ best_next, int64_t nn, const uint64_t* __restrict__ hot_count,
    Ctrl* ctrl) {
    __shared__ uint32_t s_lab[kTileArcs];
    __shared__ uint32_t s_rs[kBucketMax];
    __shared__ uint64_t s_src[kBucketMax];
    __shared__ uint32_t s_na;
    __shared__ unsigned long long s_hmin[kHotIds];   // minima of the labels below kh
    __shared__ uint64_t s_w[kPassThreads / kWave];
    const int tid = threadIdx.x;
    const uint64_t narcs = 2 * (uint64_t)m;
    uint32_t kept = 0;
    bool bad = false;
    // The hot labels were renumbered first (k_hot_*): the minima of labels
    // below kh are taken in LDS and merged once per workgroup.
    const uint32_t kh = hot_count ? (uint32_t)std::min<uint64_t>(*hot_count, (uint64_t)kHotIds) : 0u;
    for (uint32_t i = tid; i < kh; i += kPassThreads) s_hmin[i] = kKeyMax;
    // Thread bk holds bucket bk's run of the tile: its base once, the run
    // entries of the next tile loaded while this tile's edges are processed.
    static_assert(kPassThreads == kBucketMax, "one thread per bucket");
    const int bk = tid;
    const bool has_bk = bk < (int)nb;
    const uint64_t bbase = has_bk ? base[bk] : 0;
    uint32_t mt_n = 0, of_n = 0;
    // neighbouring tiles read the two ends of shared label-run lines: they go
    // to workgroups of one XCD (xcd_slot)
    const uint32_t t0 = xcd_slot(blockIdx.x, gridDim.x);
    if (has_bk && t0 < nt) {
        mt_n = meta[(int64_t)t0 * nb + bk];
        of_n = offt[(int64_t)t0 * nb + bk];
    }
    // tiles are taken grid-stride, so the live-edge count costs one atomic
    // per workgroup (same-address atomics queue at ~13 ns each)
    for (uint32_t t = t0; t < nt; t += gridDim.x) {
        const int64_t e0 = (int64_t)t << kBucketTileShift;
        const int64_t e1 = e0 + kBucketTile < m ? e0 + kBucketTile : m;
        if (has_bk) {
            s_rs[bk] = mt_n & 0xffff;
            s_src[bk] = bbase + of_n;
            if (bk == (int)nb - 1) s_na = std::min((mt_n & 0xffff) + (mt_n >> 16), (uint32_t)kTileArcs);
        } else {
            s_rs[bk] = 0xffffffffu;   // past the last bucket: never <= a slot
            s_src[bk] = 0;
        }
        __syncthreads();
        const uint32_t na = s_na;
        for (uint32_t x0 = tid; x0 < na; x0 += kInFlight * kPassThreads) {
            uint32_t val[kInFlight];
#pragma unroll
            for (int k = 0; k < kInFlight; ++k) {
                const uint32_t x = x0 + k * kPassThreads;
                val[k] = 0;
                if (x < na) {
                    const uint32_t b = last_le(s_rs, x);
                    const uint64_t i = s_src[b] + (x - s_rs[b]);
                    if (i < narcs) val[k] = __builtin_nontemporal_load(relab + i);
                }
            }
#pragma unroll
            for (int k = 0; k < kInFlight; ++k) {
                const uint32_t x = x0 + k * kPassThreads;
                if (x < na) s_lab[x] = val[k];
            }
        }
        __syncthreads();
        const uint32_t tn = t + gridDim.x;
        if (has_bk && tn < nt) {
            mt_n = meta[(int64_t)tn * nb + bk];
            of_n = offt[(int64_t)tn * nb + bk];
        }
        // the tile's edges in two parts of kGroups x 4 per lane (register budget)
        for (int part = 0; part < kPassParts; ++part) {
            const int64_t qbase = e0 / 4 + (int64_t)part * kGroups * kPassThreads + tid;
            uint32_t ww[kGroups][4], rk[kGroups][4];
#pragma unroll
            for (int j = 0; j < kGroups; ++j) {
                const int64_t q = qbase + (int64_t)j * kPassThreads;
                load4_nt(w, q, e1, ww[j]);
                load4_nt(rank, q, e1, rk[j]);
            }
            // The lane's 2 x kGroups x 4 reads of best_next are issued together,
            // then the atomics of the keys that beat them (every lane runs every step:
            // wave_min_commit needs whole waves).
            constexpr int kE = kGroups * 4;
            int32_t ra[kE], rb[kE];
            uint64_t key[kE];
            bool ax[kE], ay[kE];
#pragma unroll
            for (int j = 0; j < kGroups; ++j) {
                const int64_t q = qbase + (int64_t)j * kPassThreads;
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const int i = j * 4 + k;
                    ra[i] = rb[i] = 0;
                    key[i] = kKeyMax;
                    ax[i] = ay[i] = false;
                    const int64_t e = q * 4 + k;
                    // rank 0 (both arcs at slot 0) marks an edge the scatter
                    // skipped: a self-loop or an id out of range; a real
                    // edge's two arcs have distinct slots
                    if (e < e1 && rk[j][k] != 0) {
                        const uint32_t lx = s_lab[rk[j][k] & kArcMask];
                        const uint32_t ly = s_lab[(rk[j][k] >> 16) & kArcMask];
                        if (lx != ly) {
                            if (lx >= (uint64_t)nn || ly >= (uint64_t)nn) {
                                bad = true;
                            } else {
                                ra[i] = (int32_t)lx;
                                rb[i] = (int32_t)ly;
                                ++kept;
                                // side keys: the v end's key has bit 0 set
                                key[i] = ((uint64_t)ww[j][k] << 32) | ((uint64_t)e << 1);
                                ax[i] = lx >= kh;
                                ay[i] = ly >= kh;
                                if (!ax[i] && key[i] < s_hmin[lx])
                                    atomicMin(&s_hmin[lx], (unsigned long long)key[i]);
                                if (!ay[i] && (key[i] | 1u) < s_hmin[ly])
                                    atomicMin(&s_hmin[ly], (unsigned long long)(key[i] | 1u));
                            }
                        }
                    }
                }
                if (q * 4 < e1) store_group<OUT, true>(q, m, *reinterpret_cast<int32_t(*)[4]>(&ra[j * 4]),
                                                 *reinterpret_cast<int32_t(*)[4]>(&rb[j * 4]), ou, ov, op16);
            }
            uint64_t cx[kE], cy[kE];
#pragma unroll
            for (int i = 0; i < kE; ++i) {
                cx[i] = ax[i] ? best_next[ra[i]] : 0;
                cy[i] = ay[i] ? best_next[rb[i]] : 0;
            }
#pragma unroll
            for (int i = 0; i < kE; ++i) {
                const uint64_t kb = key[i] | 1u;
                wave_min_commit(best_next, ra[i], key[i], ax[i] && key[i] < cx[i]);
                wave_min_commit(best_next, rb[i], kb, ay[i] && kb < cy[i]);
            }
        }
        __syncthreads();   // the next tile reuses the LDS tables
    }
    for (uint32_t i = tid; i < kh; i += kPassThreads)
        if (s_hmin[i] != kKeyMax) atomic_min_key(&best_next[i], s_hmin[i]);
    uint64_t tot;
    (void)block_excl_scan(kept, s_w, &tot);
    if (tid == 0 && tot) atomicAdd((unsigned long long*)&ctrl->m_next, (unsigned long long)tot);
    if (__ballot(bad) && lane_id() == 0) atomicOr(&ctrl->err, kErrInternal);
}

// Hot-first renumbering of the round-1 labels.  After round 0 of a skewed
// graph a few thousand components carry a large share of the edge ends; the
// relabelling pass keeps the minima of the smallest kHotIds labels in LDS and
// the next pass the prefix of its label map, so the components met most
// often get the smallest labels.  kHotSample edge ends are sampled by a
// counter-based hash (SplitMix64 output function of the sample index) and
// counted per label with atomics.  The sampled labels fall into four tiers by
// count (at least 16, 4, 2, then 1); the new labels are a permutation of
// [0, nn): tier by tier, hottest first, each tier in label order, then the
// labels never sampled.  One u64 scan ranks all tiers at once: tier t adds
// 1 << 16t, and no tier holds more than kHotSample < 2^16 labels.

// cnt[l] += 1 for every sampled edge end with label l (cnt zeroed before).
__global__ __launch_bounds__(kBlock) void k_hot_count(const int32_t* __restrict__ u,
                                                      const int32_t* __restrict__ v, int64_t m,
                                                      const int32_t* __restrict__ lab,
                                                      uint64_t* __restrict__ cnt) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kHotSample) return;
    uint64_t z = (uint64_t)i * 0x9E3779B97F4A7C15ull + 0x243F6A8885A308D3ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    const int64_t e = (int64_t)__umul64hi(z, (uint64_t)m);
    const int32_t x = (i & 1) ? v[e] : u[e], y = (i & 1) ? u[e] : v[e];
    const int32_t l = x != y ? lab[x] : -1;
    // the lanes sampling the first active lane's label add once (a giant
    // component would otherwise queue one same-address atomic per sample)
    const uint64_t am = __ballot(l >= 0);
    if (am == 0) return;
    const int leader = __builtin_ctzll(am);
    const int32_t tl = __shfl(l, leader, kWave);
    const bool same = l >= 0 && l == tl;
    const uint64_t c = (uint64_t)__popcll(__ballot(same));
    if (lane_id() == leader) atomicAdd((unsigned long long*)&cnt[tl], (unsigned long long)c);
    if (l >= 0 && !same) atomicAdd((unsigned long long*)&cnt[l], 1ull);
}

static_assert(kHotSample < 65536, "a tier's rank must fit in 16 bits");

// cnt[l] <- 1 << 16t for a label of tier t, 0 for a label never sampled.
__global__ __launch_bounds__(kBlock) void k_hot_flags(uint64_t* __restrict__ cnt, int64_t nn) {
    for (int64_t l = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; l < nn;
         l += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t c = cnt[l];
        const int t = c >= 16 ? 0 : c >= 4 ? 1 : c >= 2 ? 2 : 3;
        cnt[l] = c ? 1ull << (16 * t) : 0;
    }
}

__device__ __forceinline__ uint64_t tier_sum(uint64_t p) {
    return (p & 0xffff) + ((p >> 16) & 0xffff) + ((p >> 32) & 0xffff) + (p >> 48);
}

// lab[x] <- new label of lab[x]; pre = exclusive scan of the tier flags
// (pre[nn] = the tiers' sizes).  Also pre[nn + 1] = labels sampled.
__global__ __launch_bounds__(kBlock) void k_hot_relabel(int32_t* __restrict__ lab, int64_t nr,
                                                        uint64_t* __restrict__ pre, int64_t nn) {
    const uint64_t T = pre[nn];
    const uint64_t H = tier_sum(T);
    if (blockIdx.x == 0 && threadIdx.x == 0) pre[nn + 1] = H;
    for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < nr;
         x += (int64_t)gridDim.x * blockDim.x) {
        const int32_t l = lab[x];
        if (l < 0 || l >= nn) continue;
        const uint64_t r = pre[l], d = pre[l + 1] - r;
        uint64_t nl;
        if (d) {
            const int t = (int)(__builtin_ctzll(d) >> 4);
            const uint64_t below = tier_sum(T & ((1ull << (16 * t)) - 1));   // earlier tiers
            nl = below + ((r >> (16 * t)) & 0xffff);
        } else {
            nl = H + ((uint64_t)l - tier_sum(r));
        }
        lab[x] = (int32_t)nl;
    }
}

// ctrl->aux[0] = how many of 4096 edges sampled evenly have |u - v| below the
// bucket width (ids with locality: the edge-list round 0 then hits in L2).
__global__ __launch_bounds__(kBucketThreads) void k_bk_locality(const int32_t* __restrict__ u,
                                                                const int32_t* __restrict__ v,
                                                                int64_t m, Ctrl* ctrl) {
    __shared__ uint64_t s_w[kBucketThreads / kWave];
    constexpr int kPer = kLocalitySample / kBucketThreads;
    static_assert(kPer * kBucketThreads == kLocalitySample, "whole samples per thread");
    int32_t a[kPer], b[kPer];
#pragma unroll
    for (int j = 0; j < kPer; ++j) {     // every load issued before the first compare
        const uint64_t k = (uint64_t)(threadIdx.x + j * kBucketThreads);
        const int64_t e = (int64_t)((k * (uint64_t)m) / kLocalitySample);
        a[j] = u[e];
        b[j] = v[e];
    }
    uint64_t local = 0;
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        const int64_t d = (int64_t)a[j] - (int64_t)b[j];
        local += (d < kBucketWidth && -d < kBucketWidth) ? 1 : 0;
    }
    uint64_t tot;
    (void)block_excl_scan(local, s_w, &tot);
    if (threadIdx.x == 0) ctrl->aux[0] = tot;
}

// -------------------------------------------------------------- launchers

void bucket_hot_first(const BucketBuffers& B, const int32_t* u, const int32_t* v, int64_t m,
                      int32_t* lab, int64_t nr, int64_t nn, hipStream_t s) {
    const int h = prof_begin(K_BK_INDEX, s);
    B.hotn = nn;
    launch_fill_u64(B.hotpre, nn + 1, 0, s);
    hipLaunchKernelGGL(k_hot_count, dim3((kHotSample + kBlock - 1) / kBlock), dim3(kBlock), 0, s, u,
                       v, m, lab, B.hotpre);
    hipLaunchKernelGGL(k_hot_flags, dim3((unsigned)std::min<int64_t>((nn + kBlock - 1) / kBlock, 4096)),
                       dim3(kBlock), 0, s, B.hotpre, nn);
    launch_scan_u64(B.hotpre, nn, B.hottmp, B.hotpre + nn, s);
    const int64_t g = std::min<int64_t>((nr + kBlock - 1) / kBlock, 4096);
    hipLaunchKernelGGL(k_hot_relabel, dim3((unsigned)g), dim3(kBlock), 0, s, lab, nr, B.hotpre, nn);
    prof_end(h, s, 8.0 * nr + 24.0 * nn);
}

void bucket_sample_locality(const int32_t* u, const int32_t* v, int64_t m, Ctrl* ctrl,
                            hipStream_t s) {
    hipLaunchKernelGGL(k_bk_locality, dim3(1), dim3(kBucketThreads), 0, s, u, v, m, ctrl);
}

static unsigned transpose_grid(int64_t R, int64_t C) {
    return (unsigned)(((R + 31) / 32) * ((C + 31) / 32));
}

void bucket_minedge(const BucketBuffers& B, const int32_t* u, const int32_t* v,
                    const uint32_t* w, int64_t m, int64_t n, uint64_t* best, Ctrl* ctrl,
                    hipStream_t s) {
    const uint32_t nb = (uint32_t)nbuckets(n), nt = (uint32_t)ntiles(m);
    const double cells = (double)nb * nt, arcs = 2.0 * (double)m;
    const dim3 bl(kBucketThreads);
    B.hotn = -1;   // no hot-first renumbering yet in this solve
    int h = prof_begin(K_BK_SCATTER, s);
    hipLaunchKernelGGL(k_bk_scatter, dim3(std::min<uint32_t>(nt, kScatterGrid)), bl, 0, s, u, v,
                       w, m, n, nb, nt, B.arcs, B.meta, B.rank, ctrl);
    prof_end(h, s, 12.0 * m + 8.0 * arcs + 4.0 * m + 4.0 * cells);
    h = prof_begin(K_BK_INDEX, s);
    hipLaunchKernelGGL(k_transpose_u32, dim3(transpose_grid(nt, nb)), dim3(256), 0, s, B.meta,
                       B.metat, (int64_t)nt, (int64_t)nb);
    hipLaunchKernelGGL(k_bk_totals, dim3(nb), dim3(256), 0, s, B.metat, nt, B.base);
    launch_scan_u64(B.base, nb, B.tmp, B.base + nb, s);
    prof_end(h, s, 12.0 * cells + 24.0 * nb);
    h = prof_begin(K_BK_MIN, s);
    hipLaunchKernelGGL(k_bk_min, dim3(nb), bl, 0, s, B.arcs, B.metat, nt, n, 2 * m, B.base, best,
                       B.xs, B.offb);
    prof_end(h, s, 8.0 * arcs + 2.0 * arcs + 8.0 * cells + 8.0 * n);
    h = prof_begin(K_BK_INDEX, s);
    hipLaunchKernelGGL(k_transpose_u32, dim3(transpose_grid(nb, nt)), dim3(256), 0, s, B.offb,
                       B.offt, (int64_t)nb, (int64_t)nt);
    prof_end(h, s, 8.0 * cells);
}

void bucket_relabel(const BucketBuffers& B, const uint32_t* w, int64_t m, int64_t n,
                    const int32_t* M, int out,
                    int32_t* ou, int32_t* ov, uint32_t* op16, uint64_t* best_next, int64_t nn,
                    Ctrl* ctrl, hipStream_t s) {
    const uint32_t nb = (uint32_t)nbuckets(n), nt = (uint32_t)ntiles(m);
    const double cells = (double)nb * nt, arcs = 2.0 * (double)m;
    uint32_t* relab = reinterpret_cast<uint32_t*>(B.arcs);
    const dim3 bl(kBucketThreads);
    int h = prof_begin(K_BK_LABEL, s);
    hipLaunchKernelGGL(k_bk_label, dim3(nb), bl, 0, s, B.xs, B.base, n, 2 * m, M, relab);
    prof_end(h, s, 6.0 * arcs + 4.0 * n);
    // the count of renumbered hot labels, if this solve renumbered them
    const uint64_t* hot_count = B.hotn >= 0 && B.hotn <= nn ? B.hotpre + B.hotn + 1 : nullptr;
    h = prof_begin(K_BK_PASS, s);
    const dim3 grid(std::min<uint32_t>(nt, kPassGrid)), pbl(kPassThreads);
    if (out == kOut16)
        hipLaunchKernelGGL(k_bk_pass<kOut16>, grid, pbl, 0, s, w, m, nb, nt, B.meta,
                           B.offt, B.base, relab, B.rank, ou, ov, op16, best_next, nn, hot_count, ctrl);
    else
        hipLaunchKernelGGL(k_bk_pass<kOut32>, grid, pbl, 0, s, w, m, nb, nt, B.meta,
                           B.offt, B.base, relab, B.rank, ou, ov, op16, best_next, nn, hot_count, ctrl);
    prof_end(h, s, 8.0 * m + 4.0 * arcs + (out == kOut16 ? 4.0 : 8.0) * m + 8.0 * cells +
                       8.0 * nn);
}

}  // namespace msf
