// Filter-Borůvka (paper Sec. V, Alg. 2) on one GPU.
//
//   Rec-Filter-MST(E):
//     if isSparse(E): Borůvka base case on E, recording representatives in P
//     pivot  <- sample quantile of the keys of E            (PivotSelection)
//     E<=, E> <- stable split of E by key <= pivot
//     Rec-Filter-MST(E<=)
//     E>'    <- {(P[u], P[v]) : (u, v) in E>, P[u] != P[v]} (Filter)
//     Rec-Filter-MST(E>')
//
// Keys are (w << 32 | edge id); comparing whole keys (not only weights) keeps
// the split proper even when many weights tie.  Every layout keeps edges in
// id order, so the base case may again use positions as tie-break keys.
#include <string.h>

#include <algorithm>

#include "filter.h"
#include "mlp.h"
#include "prim.h"

namespace msf {

namespace {
constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ULL;
constexpr uint64_t kPivotTag = 0x50495654ULL;   // stream tag of the pivot sampler
constexpr int kSampleMax = 8192;
constexpr int kEndSample = 2048;      // sampled edges whose endpoints feed feature 14
constexpr int kSampleThreads = 1024;
constexpr int kMaxDepth = 48;
}  // namespace

// SplitMix64 output function (Steele, Lea & Flood, OOPSLA 2014).
__host__ __device__ __forceinline__ uint64_t sm_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

// Draw `attempt` of split `split`: the first uses mix(mix(seed) ^ (tag + split)),
// a redraw a >= 1 (balanced-split retry) mix(that + a * gamma).
uint64_t pivot_stream_base(uint64_t seed, uint32_t split, uint32_t attempt) {
    const uint64_t b = sm_mix(sm_mix(seed) ^ (kPivotTag + split));
    return attempt == 0 ? b : sm_mix(b + (uint64_t)attempt * kGamma);
}

// ------------------------------------------------------------------ kernels

__global__ void k_iota(int32_t* __restrict__ p, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = (int32_t)i;
}

template <int MODE>
__device__ __forceinline__ uint64_t key_at(const View& g, int64_t p) {
    const uint64_t id = MODE == kCompact ? (uint64_t)g.id[p] : (uint64_t)p;
    return ((uint64_t)g.w[p] << 32) | id;
}

// Pivot selection: `sample` keys drawn with replacement at positions
// floor(r_i * len / 2^64), r_i the i-th output of the counter-based stream
// `base`; bitonic sort in LDS; pivot = sorted[floor(q * (sample - 1))].
// One workgroup.  With a pivot network (`mlp` non-null) q is its output on
// features of the sorted sample, clamped to [2^-10, 1 - 2^-10] (a non-finite
// output falls back to the median); otherwise q is the argument.  The
// features are always written to ctrl->feat:
//   0-4   L(w) at the 10/25/50/75/90 % sample quantiles, L(w) = log2(1+w)/32
//   5, 6  mean and standard deviation of L over the sample
//   7     fraction of adjacent equal weights in the sorted sample (ties)
//   8, 9  L of the smallest and largest sampled weight
//   10    log2(1 + current components) / 32
//   11    log2(1 + edges of this graph) / 32
//   12    log2(1 + edges / components) / 8
//   13    recursion depth / 16
//   14    fraction of repeated endpoints among the first <= 2048 sampled
//         edges (a degree-skew proxy)
//   15    1
// One compare-exchange stage of an ascending bitonic sort of a[0, n) in LDS.
template <typename T>
__device__ __forceinline__ void bitonic_stage(T* a, int n, int k, int j) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const int ixj = i ^ j;
        if (ixj > i) {
            const T x = a[i], y = a[ixj];
            if ((x > y) == ((i & k) == 0)) { a[i] = y; a[ixj] = x; }
        }
    }
}

// Ascending bitonic sort of a[0, kRegSort) in LDS by the whole workgroup:
// thread t keeps elements 4t .. 4t + 3 in registers.  Stages whose partner is
// in the same thread run in registers, those with a partner in another lane
// of the wave by lane shuffles, and only the stages that cross waves (partner
// distance >= 4 * kWave) go through LDS, with workgroup barriers.
constexpr int kRegSort = 4 * kSampleThreads;
template <typename T>
__device__ __forceinline__ void cmpx(T& a, T& b, bool up) {
    if ((a > b) == up) { const T t = a; a = b; b = t; }
}
template <typename T>
__device__ __forceinline__ void bitonic_sort_regs(T* a) {
    const int t = threadIdx.x;
    T x[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) x[r] = a[4 * t + r];
    for (int k = 2; k <= kRegSort; k <<= 1) {
        int j = k >> 1;
        if (j >= 4 * kWave) {                      // partners in other waves: LDS
#pragma unroll
            for (int r = 0; r < 4; ++r) a[4 * t + r] = x[r];
            __syncthreads();
            for (; j >= 4 * kWave; j >>= 1) {
                bitonic_stage(a, kRegSort, k, j);
                __syncthreads();
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) x[r] = a[4 * t + r];
        }
        for (; j >= 4; j >>= 1) {                  // partner in lane t ^ (j / 4)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = 4 * t + r;
                const T y = __shfl_xor(x[r], j / 4, kWave);
                const bool keep_min = ((i & j) == 0) == ((i & k) == 0);
                x[r] = keep_min ? (y < x[r] ? y : x[r]) : (y < x[r] ? x[r] : y);
            }
        }
        const bool up0 = ((4 * t) & k) == 0, up2 = ((4 * t + 2) & k) == 0;
        if (j == 2) {                              // partners in this thread
            cmpx(x[0], x[2], up0);
            cmpx(x[1], x[3], up0);
            j = 1;
        }
        cmpx(x[0], x[1], up0);
        cmpx(x[2], x[3], up2);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) a[4 * t + r] = x[r];
}

template <int MODE>
__global__ __launch_bounds__(kSampleThreads) void k_sample_pivot(View g, uint64_t base,
                                                                 int sample, float q,
                                                                 const float* __restrict__ mlp,
                                                                 float comps, int depth,
                                                                 Ctrl* ctrl) {
    __shared__ uint64_t keys[kSampleMax];
    __shared__ int32_t ends[kEndSample * 2];
    __shared__ float red[2 * kSampleThreads / kWave];
    __shared__ float feat[kMlpIn];
    __shared__ float hid[2 * kMlpH];
    __shared__ uint32_t s_cnt[2];
    int p2 = 1;
    while (p2 < sample) p2 <<= 1;
    const int ke = sample < kEndSample ? sample : kEndSample;
    int e2 = 1;
    while (e2 < 2 * ke) e2 <<= 1;
    const uint64_t len = (uint64_t)g.len;
    if (threadIdx.x < 2) s_cnt[threadIdx.x] = 0;
    for (int i = threadIdx.x; i < p2; i += blockDim.x) {
        uint64_t k = kKeyMax;
        if (i < sample) {
            const uint64_t r = sm_mix(base + (uint64_t)(i + 1) * kGamma);
            const int64_t pos = (int64_t)__umul64hi(r, len);
            k = key_at<MODE>(g, pos);
            if (i < ke) {
                ends[2 * i] = g.u[pos];
                ends[2 * i + 1] = g.v[pos];
            }
        }
        keys[i] = k;
    }
    for (int i = 2 * ke + threadIdx.x; i < e2; i += blockDim.x) ends[i] = 0x7fffffff;
    __syncthreads();
    // Both arrays are sorted together.  In a stage with j < 64 the pair
    // (i, i ^ j) belongs to one wave (thread t handles i = t mod blockDim), so
    // only stages that cross waves, and the stages right before them, need the
    // workgroup barrier; the others only drain the wave's LDS operations.
    const int kmax = p2 > e2 ? p2 : e2;
    if (p2 == kRegSort && e2 == kRegSort) {          // the default sample of 4096
        bitonic_sort_regs(keys);
        bitonic_sort_regs(ends);
    } else {
        for (int k = 2; k <= kmax; k <<= 1) {
            for (int j = k >> 1; j > 0; j >>= 1) {
                if (k <= p2) bitonic_stage(keys, p2, k, j);
                if (k <= e2) bitonic_stage(ends, e2, k, j);
                const int next_j = j > 1 ? j >> 1 : k;   // first stage of the next k is j = k
                if (j >= kWave || next_j >= kWave) __syncthreads();
                else asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
            }
        }
    }
    __syncthreads();
    // sample statistics (FP32)
    float sl = 0.f, sl2 = 0.f;
    uint32_t ties = 0, reps = 0;
    for (int i = threadIdx.x; i < sample; i += blockDim.x) {
        const float l = __log2f(1.f + (float)(keys[i] >> 32)) * (1.f / 32.f);
        sl += l;
        sl2 += l * l;
        if (i + 1 < sample && (keys[i] >> 32) == (keys[i + 1] >> 32)) ++ties;
    }
    for (int i = threadIdx.x; i + 1 < 2 * ke; i += blockDim.x) reps += ends[i] == ends[i + 1];
    for (int off = 32; off > 0; off >>= 1) {
        sl += __shfl_xor(sl, off, 64);
        sl2 += __shfl_xor(sl2, off, 64);
    }
    const int wv = threadIdx.x / kWave;
    if (lane_id() == 0) { red[wv] = sl; red[kSampleThreads / kWave + wv] = sl2; }
    if (ties) atomicAdd(&s_cnt[0], ties);
    if (reps) atomicAdd(&s_cnt[1], reps);
    __syncthreads();
    if (threadIdx.x == 0) {
        float a = 0.f, b = 0.f;
        for (int i = 0; i < kSampleThreads / kWave; ++i) { a += red[i]; b += red[kSampleThreads / kWave + i]; }
        const float mean = a / (float)sample;
        const float var = b / (float)sample - mean * mean;
        const float qs[5] = {0.1f, 0.25f, 0.5f, 0.75f, 0.9f};
        for (int k = 0; k < 5; ++k) {
            const int idx = (int)(qs[k] * (float)(sample - 1));
            feat[k] = __log2f(1.f + (float)(keys[idx] >> 32)) * (1.f / 32.f);
        }
        feat[5] = mean;
        feat[6] = sqrtf(var > 0.f ? var : 0.f);
        feat[7] = sample > 1 ? (float)s_cnt[0] / (float)(sample - 1) : 0.f;
        feat[8] = __log2f(1.f + (float)(keys[0] >> 32)) * (1.f / 32.f);
        feat[9] = __log2f(1.f + (float)(keys[sample - 1] >> 32)) * (1.f / 32.f);
        feat[10] = __log2f(1.f + comps) * (1.f / 32.f);
        feat[11] = __log2f(1.f + (float)len) * (1.f / 32.f);
        feat[12] = __log2f(1.f + (float)len / (comps > 1.f ? comps : 1.f)) * (1.f / 8.f);
        feat[13] = (float)depth * (1.f / 16.f);
        feat[14] = 2 * ke > 1 ? (float)s_cnt[1] / (float)(2 * ke - 1) : 0.f;
        feat[15] = 1.f;
        for (int k = 0; k < kMlpIn; ++k) ctrl->feat[k] = feat[k];
    }
    __syncthreads();
    float qq = q;
    if (mlp) {
        const float z = mlp_infer_block(mlp, feat, hid);
        const float p = 1.f / (1.f + expf(-z));
        qq = (p == p) ? fminf(fmaxf(p, kQMin), 1.f - kQMin) : 0.5f;
    }
    if (threadIdx.x == 0) {
        int idx = (int)floor((double)qq * (double)(sample - 1));
        if (idx < 0) idx = 0;
        if (idx > sample - 1) idx = sample - 1;
        ctrl->pivot = keys[idx];
        ctrl->q_used = qq;
    }
}

// Split counts, reduce-then-scan: the light-edge count (key <= pivot) of
// every 2048-edge tile goes to cnt[tile]; k_scan_tiles turns the counts into
// exclusive offsets, so the split pass needs no inter-tile waiting.  One wave
// per tile: lane l reads 4 consecutive edges at l*4 + j*256 (j < 8) with
// 16-byte loads when the arrays allow it, so no workgroup barrier is needed.
template <int MODE, bool VEC>
__global__ __launch_bounds__(kBlock) void k_count_tiles(View g,
                                                        const uint64_t* __restrict__ pivot_dev,
                                                        uint64_t* __restrict__ cnt,
                                                        uint32_t ntiles) {
    const uint64_t pivot = *pivot_dev;
    const int lane = threadIdx.x % kWave;
    const uint32_t waves = gridDim.x * (kBlock / kWave);
    for (uint32_t t = blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave; t < ntiles;
         t += waves) {
        const int64_t e0 = (int64_t)t * kRelabelTile;
        uint32_t c = 0;
        if (VEC && e0 + kRelabelTile <= g.len) {
            uint4 wv[kRelabelTile / 256], iv[kRelabelTile / 256];
#pragma unroll
            for (int j = 0; j < kRelabelTile / 256; ++j) {
                const int64_t q = (e0 + j * 256 + lane * 4) / 4;
                wv[j] = reinterpret_cast<const uint4*>(g.w)[q];
                iv[j] = MODE == kCompact ? reinterpret_cast<const uint4*>(g.id)[q]
                                         : make_uint4(0, 0, 0, 0);
            }
#pragma unroll
            for (int j = 0; j < kRelabelTile / 256; ++j) {
                const uint64_t e = (uint64_t)(e0 + j * 256 + lane * 4);
                const uint32_t ws[4] = {wv[j].x, wv[j].y, wv[j].z, wv[j].w};
                const uint32_t is[4] = {iv[j].x, iv[j].y, iv[j].z, iv[j].w};
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const uint64_t id = MODE == kCompact ? (uint64_t)is[i] : e + i;
                    c += (((uint64_t)ws[i] << 32) | id) <= pivot;
                }
            }
        } else {
            for (int64_t e = e0 + lane; e < e0 + kRelabelTile && e < g.len; e += kWave) {
                const uint64_t id = MODE == kCompact ? (uint64_t)g.id[e] : (uint64_t)e;
                c += (((uint64_t)g.w[e] << 32) | id) <= pivot;
            }
        }
        for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off, kWave);
        if (lane == 0) cnt[t] = c;
    }
}

// Workgroups of the tile kernels (split, filter): each loops over tiles, so a
// launch is not dominated by dispatching one short workgroup per tile.
constexpr unsigned kTileGrid = 4096;
// Exclusive scan of the tile counts cnt[0, nt) in place, in three short
// launches: per-chunk sums (kScanChunk counts per workgroup), one workgroup
// scanning the <= kScanTop chunk sums (and writing the total), per-chunk
// scans offset by their chunk's prefix.
constexpr int kScanChunk = kBlock * 8;
constexpr int kScanTop = 1024;     // chunk sums: nt <= 2^21 tiles covers m < 2^32

__global__ __launch_bounds__(kBlock) void k_scan_up(const uint64_t* __restrict__ cnt, uint32_t nt,
                                                    uint64_t* __restrict__ bsum) {
    __shared__ uint64_t s_w[kBlock / kWave];
    const int64_t i0 = (int64_t)blockIdx.x * kScanChunk + threadIdx.x;
    uint64_t x = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k)
        if (i0 + k * kBlock < nt) x += cnt[i0 + k * kBlock];
    uint64_t tot;
    (void)block_excl_scan(x, s_w, &tot);
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kScanTop) void k_scan_top(uint64_t* __restrict__ bsum, uint32_t nb,
                                                       uint64_t* __restrict__ total) {
    __shared__ uint64_t s_w[kScanTop / kWave];
    const uint64_t x = threadIdx.x < nb ? bsum[threadIdx.x] : 0;
    uint64_t tot;
    const uint64_t ex = block_excl_scan(x, s_w, &tot);
    if (threadIdx.x < nb) bsum[threadIdx.x] = ex;
    if (threadIdx.x == 0) *total = tot;
}

__global__ __launch_bounds__(kBlock) void k_scan_down(uint64_t* __restrict__ cnt, uint32_t nt,
                                                      const uint64_t* __restrict__ bsum) {
    __shared__ uint64_t s_w[kBlock / kWave];
    const int64_t i0 = (int64_t)blockIdx.x * kScanChunk + (int64_t)threadIdx.x * 8;
    uint64_t c[8], x = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        c[k] = i0 + k < nt ? cnt[i0 + k] : 0;
        x += c[k];
    }
    uint64_t tot;
    uint64_t run = bsum[blockIdx.x] + block_excl_scan(x, s_w, &tot);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        if (i0 + k < nt) cnt[i0 + k] = run;
        run += c[k];
    }
}

// Exclusive scan of cnt[0, nt) in place; the sum goes to *total (device).
void launch_scan_tiles(uint64_t* cnt, uint32_t nt, uint64_t* bsum, uint64_t* total,
                       hipStream_t s) {
    const uint32_t nb = (nt + kScanChunk - 1) / kScanChunk;
    hipLaunchKernelGGL(k_scan_up, dim3(nb), dim3(kBlock), 0, s, cnt, nt, bsum);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kScanTop), 0, s, bsum, nb, total);
    hipLaunchKernelGGL(k_scan_down, dim3(nb), dim3(kBlock), 0, s, cnt, nt, bsum);
}

// Exclusive scan of cnt[0, n) in place for any n < 2^32: the chunk sums are
// scanned by one workgroup when there are at most kScanTop of them, else by
// the same three steps one level up (tmp holds every level's chunk sums:
// scan_levels_bytes(n) bytes).
size_t scan_levels_bytes(int64_t n) {
    size_t words = 0;
    for (int64_t k = n; k > 1;) {
        k = (k + kScanChunk - 1) / kScanChunk;
        words += (size_t)k;
    }
    return (words + 1) * 8;
}
void launch_scan_u64(uint64_t* cnt, int64_t n, uint64_t* tmp, uint64_t* total, hipStream_t s) {
    const uint32_t nb = (uint32_t)((n + kScanChunk - 1) / kScanChunk);
    hipLaunchKernelGGL(k_scan_up, dim3(nb), dim3(kBlock), 0, s, cnt, (uint32_t)n, tmp);
    if (nb <= (uint32_t)kScanTop)
        hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kScanTop), 0, s, tmp, nb, total);
    else
        launch_scan_u64(tmp, nb, tmp + nb, total, s);
    hipLaunchKernelGGL(k_scan_down, dim3(nb), dim3(kBlock), 0, s, cnt, (uint32_t)n, tmp);
}

// Stable two-way split by key <= pivot: tile t writes its light edges from
// off[t] on and its heavy edges from nl' + (t * 2048 - off[t]) on, where
// nl' = ctrl->light rounded up to a multiple of 4 (both parts start 16-byte
// aligned).  LIGHT_ONLY writes the light part only (the heavy edges are then
// read where they are, in the caller's arrays).  On the caller's arrays the
// ids are validated.
template <int MODE, bool LIGHT_ONLY>
__global__ __launch_bounds__(kBlock) void k_split(View g, int64_t n,
                                                  const uint64_t* __restrict__ pivot_dev,
                                                  EdgeSoA out,
                                                  const uint64_t* __restrict__ tile_off,
                                                  Ctrl* ctrl, uint32_t ntiles) {
    constexpr int kIt = kRelabelItems;
    __shared__ uint32_t s_wave[kBlock / kWave];
    const uint64_t pivot = *pivot_dev;
    const uint64_t nl_al = (ctrl->light + 3) & ~3ull;
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    for (uint32_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int64_t e0 = (int64_t)tile * (kBlock * kIt) + (int64_t)wave * (kWave * kIt) + lane;
        const int64_t m = g.len;
        int32_t a[kIt], b[kIt];
        uint32_t w[kIt], idv[kIt];
        uint64_t mk[kIt];
        uint32_t cnt = 0;
        bool bad = false;
#pragma unroll
        for (int k = 0; k < kIt; ++k) {
            const int64_t e = e0 + k * kWave;
            a[k] = b[k] = 0;
            w[k] = idv[k] = 0;
            bool lt = false;
            if (e < m) {
                a[k] = g.u[e];
                b[k] = g.v[e];
                w[k] = g.w[e];
                idv[k] = MODE == kCompact ? g.id[e] : (uint32_t)e;
                if (MODE == kOrig && ((uint32_t)a[k] >= (uint64_t)n || (uint32_t)b[k] >= (uint64_t)n)) {
                    bad = true;
                    a[k] = b[k] = 0;
                }
                const uint64_t id = MODE == kCompact ? (uint64_t)idv[k] : (uint64_t)e;
                lt = (((uint64_t)w[k] << 32) | id) <= pivot;
            }
            mk[k] = __ballot(lt);
            cnt += __popcll(mk[k]);
        }
        if (__ballot(bad) && lane == 0) atomicOr(&ctrl->err, kErrRange);
        if (lane == 0) s_wave[wave] = cnt;
        __syncthreads();
        uint32_t woff = 0;
#pragma unroll
        for (int i = 0; i < kBlock / kWave; ++i)
            if (i < wave) woff += s_wave[i];
        uint64_t off = tile_off[tile] + woff;
#pragma unroll
        for (int k = 0; k < kIt; ++k) {
            const int64_t e = e0 + k * kWave;
            if (e < m && (!LIGHT_ONLY || ((mk[k] >> lane) & 1))) {
                const uint64_t before = off + lanes_below(mk[k]);   // light edges before e
                const uint64_t o = ((mk[k] >> lane) & 1) ? before : nl_al + ((uint64_t)e - before);
                out.u[o] = a[k];
                out.v[o] = b[k];
                out.w[o] = w[k];
                out.id[o] = idv[k];
            }
            off += __popcll(mk[k]);
        }
        __syncthreads();                      // s_wave is reused by the next tile
    }
}

// ------------------------------------------------------------------ filter

// Largest component among kGiantSample evenly spaced vertices (P must be
// fully compressed): ctrl->giant = its representative if it holds at least
// 1/16 of the sample, else -1.  One workgroup.
constexpr int kGiantSample = 1024;
constexpr int kGiantThreads = 1024;
__global__ __launch_bounds__(kGiantThreads) void k_giant_pick(const int32_t* __restrict__ P,
                                                              int64_t n, Ctrl* ctrl) {
    __shared__ int32_t s[kGiantSample];
    __shared__ unsigned long long s_best;
    if (threadIdx.x == 0) s_best = 0;
    for (int i = threadIdx.x; i < kGiantSample; i += blockDim.x)
        s[i] = P[((int64_t)(2 * i + 1) * n) / (2 * kGiantSample)];
    __syncthreads();
    for (int k = 2; k <= kGiantSample; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < kGiantSample; i += blockDim.x) {
                const int ixj = i ^ j;
                if (ixj > i) {
                    const int32_t a = s[i], b = s[ixj];
                    if ((a > b) == ((i & k) == 0)) { s[i] = b; s[ixj] = a; }
                }
            }
            __syncthreads();
        }
    }
    for (int i = threadIdx.x; i < kGiantSample; i += blockDim.x) {
        if (i > 0 && s[i] == s[i - 1]) continue;
        int lo = i, hi = kGiantSample;   // end of the run of s[i]
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (s[mid] <= s[i]) lo = mid + 1;
            else hi = mid;
        }
        atomicMax(&s_best, ((unsigned long long)(lo - i) << 32) | (uint32_t)s[i]);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t len = (uint32_t)(s_best >> 32);
        ctrl->giant = 16 * len >= (uint32_t)kGiantSample ? (int32_t)(uint32_t)s_best : -1;
    }
}

// Bits 0, 1, 2, ... of x at bit positions 0, 2, 4, ... (32 -> 64 bits).
__device__ __forceinline__ uint64_t spread_bits(uint64_t x) {
    x &= 0xffffffffull;
    x = (x | (x << 16)) & 0x0000ffff0000ffffull;
    x = (x | (x << 8)) & 0x00ff00ff00ff00ffull;
    x = (x | (x << 4)) & 0x0f0f0f0f0f0f0f0full;
    x = (x | (x << 2)) & 0x3333333333333333ull;
    x = (x | (x << 1)) & 0x5555555555555555ull;
    return x;
}

// 2-bit representative code of every vertex, 32 vertices per word:
// bit 0 = P[x] is ctrl->giant, bit 1 = P[x] == x; 0 = look P[x] up.
__global__ __launch_bounds__(kBlock) void k_rep_codes(const int32_t* __restrict__ P, int64_t n,
                                                      const Ctrl* ctrl,
                                                      uint64_t* __restrict__ codes) {
    const int32_t gi = ctrl->giant;
    const int64_t chunks = (n + 63) / 64;
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x / kWave);
    const int lane = threadIdx.x % kWave;
    for (int64_t c = blockIdx.x * (int64_t)(blockDim.x / kWave) + threadIdx.x / kWave; c < chunks;
         c += waves) {
        const int64_t x = c * 64 + lane;
        const int32_t p = x < n ? P[x] : -1;
        const uint64_t g = __ballot(gi >= 0 && p == gi);
        const uint64_t self = __ballot(x < n && p == (int32_t)x);
        if (lane < 2) {
            const int sh = 32 * lane;
            codes[2 * c + lane] = spread_bits(g >> sh) | (spread_bits(self >> sh) << 1);
        }
    }
}

// Representative of x from its code (one gather only for code 0).
__device__ __forceinline__ int32_t rep_of(const uint64_t* __restrict__ codes,
                                          const int32_t* __restrict__ P, int32_t gi, int32_t x) {
    const uint32_t c = (uint32_t)(codes[(uint32_t)x >> 5] >> (2 * ((uint32_t)x & 31))) & 3u;
    return (c & 1u) ? gi : (c ? x : P[x]);
}

// Filter, pass 1: keep flag of every heavy edge (flags, one bit per edge, word
// i covering edges [64i, 64i + 64)) and the kept count of every 2048-edge tile.
// An edge is dropped when both ends have the same representative; the 2-bit
// codes resolve most ends (largest component, own representative) without
// reading P.  ORIG: g is the caller's arrays, of which the heavy edges are
// those with key (w << 32 | position) > pivot; otherwise every edge of g is
// heavy.
template <bool ORIG>
__global__ __launch_bounds__(kBlock) void k_filter_flags(View g, const int32_t* __restrict__ P,
                                                         const uint64_t* __restrict__ codes,
                                                         const Ctrl* ctrl, uint64_t pivot,
                                                         uint64_t* __restrict__ flags,
                                                         uint64_t* __restrict__ cnt,
                                                         uint32_t ntiles) {
    constexpr int kIt = kRelabelItems;
    __shared__ uint32_t s_wave[kBlock / kWave];
    const int32_t gi = ctrl->giant;
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    for (uint32_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int64_t w0 = (int64_t)tile * (kBlock * kIt / kWave) + wave * kIt;  // first flag word
        const int64_t m = g.len;
        // the edges are streamed once: non-temporal loads keep the codes in the L2
        int32_t a[kIt], b[kIt];
#pragma unroll
        for (int k = 0; k < kIt; ++k) {
            const int64_t e = (w0 + k) * kWave + lane;
            a[k] = b[k] = 0;
            if (e < m) { a[k] = __builtin_nontemporal_load(g.u + e); b[k] = __builtin_nontemporal_load(g.v + e); }
            if (ORIG && e < m &&
                (((uint64_t)__builtin_nontemporal_load(g.w + e) << 32) | (uint64_t)e) <= pivot)
                b[k] = a[k];                  // light: already handled, never kept
        }
        // all code words first, then the P gathers of ends with code 0, then
        // the ballots: the lookups of a thread's edges overlap
        uint64_t ca[kIt], cb[kIt];
#pragma unroll
        for (int k = 0; k < kIt; ++k) {
            ca[k] = cb[k] = 0;
            if (a[k] != b[k]) {
                ca[k] = codes[(uint32_t)a[k] >> 5];
                cb[k] = codes[(uint32_t)b[k] >> 5];
            }
        }
        int32_t ra[kIt], rb[kIt];
#pragma unroll
        for (int k = 0; k < kIt; ++k) {
            ra[k] = rb[k] = 0;
            if (a[k] == b[k]) continue;
            const uint32_t xa = (uint32_t)(ca[k] >> (2 * ((uint32_t)a[k] & 31))) & 3u;
            const uint32_t xb = (uint32_t)(cb[k] >> (2 * ((uint32_t)b[k] & 31))) & 3u;
            ra[k] = (xa & 1u) ? gi : (xa ? a[k] : P[a[k]]);
            rb[k] = (xb & 1u) ? gi : (xb ? b[k] : P[b[k]]);
        }
        uint32_t c = 0;
#pragma unroll
        for (int k = 0; k < kIt; ++k) {
            const bool keep = a[k] != b[k] && ra[k] != rb[k];
            const uint64_t mk = __ballot(keep);
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
        __syncthreads();                      // s_wave is reused by the next tile
    }
}

// Filter, pass 2: the kept edges, relabelled (P[u], P[v]), in their order to
// out[0, kept); tile t starts at off[t] (exclusive scan of the tile counts).
// ORIG: ids are positions in the caller's arrays.
template <bool ORIG>
__global__ __launch_bounds__(kBlock) void k_filter_scatter(View g, const int32_t* __restrict__ P,
                                                           const uint64_t* __restrict__ codes,
                                                           const Ctrl* ctrl,
                                                           const uint64_t* __restrict__ flags,
                                                           const uint64_t* __restrict__ tile_off,
                                                           EdgeSoA out, uint32_t ntiles) {
    constexpr int kIt = kRelabelItems;
    __shared__ uint32_t s_wave[kBlock / kWave];
    const int32_t gi = ctrl->giant;
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int64_t words = (g.len + kWave - 1) / kWave;
    for (uint32_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int64_t w0 = (int64_t)tile * (kBlock * kIt / kWave) + wave * kIt;
        uint64_t mk[kIt];
        uint32_t c = 0;
#pragma unroll
        for (int k = 0; k < kIt; ++k) {
            mk[k] = w0 + k < words ? flags[w0 + k] : 0;
            c += __popcll(mk[k]);
        }
        if (lane == 0) s_wave[wave] = c;
        __syncthreads();
        uint32_t woff = 0;
#pragma unroll
        for (int i = 0; i < kBlock / kWave; ++i)
            if (i < wave) woff += s_wave[i];
        const uint64_t off = tile_off[tile] + woff;
        // all loads first, then the representative lookups, then the stores:
        // the kept edges of a tile are scattered, so every step is a gather
        // and the chains must overlap rather than run one after another
        int32_t a[kIt], b[kIt];
        uint32_t wt[kIt], id[kIt];
#pragma unroll
        for (int k = 0; k < kIt; ++k) {
            a[k] = b[k] = 0;
            wt[k] = id[k] = 0;
            if ((mk[k] >> lane) & 1) {   // read once: non-temporal, the codes stay in the L2
                const int64_t e = (w0 + k) * kWave + lane;
                a[k] = __builtin_nontemporal_load(g.u + e);
                b[k] = __builtin_nontemporal_load(g.v + e);
                wt[k] = __builtin_nontemporal_load(g.w + e);
                id[k] = ORIG ? (uint32_t)e : __builtin_nontemporal_load(g.id + e);
            }
        }
#pragma unroll
        for (int k = 0; k < kIt; ++k) {
            if ((mk[k] >> lane) & 1) {
                a[k] = rep_of(codes, P, gi, a[k]);
                b[k] = rep_of(codes, P, gi, b[k]);
            }
        }
        uint64_t o = off;
#pragma unroll
        for (int k = 0; k < kIt; ++k) {
            if ((mk[k] >> lane) & 1) {
                const uint64_t d = o + lanes_below(mk[k]);
                out.u[d] = a[k];
                out.v[d] = b[k];
                out.w[d] = wt[k];
                out.id[d] = id[k];
            }
            o += __popcll(mk[k]);
        }
        __syncthreads();                      // s_wave is reused by the next tile
    }
}

// ---------------------------------------------------------------- launchers

static inline unsigned grid_cap(int64_t n, unsigned cap = 2048) {
    int64_t g = (n + kBlock - 1) / kBlock;
    if (g < 1) g = 1;
    return (unsigned)(g < cap ? g : cap);
}

void launch_iota(int32_t* p, int64_t n, hipStream_t s) {
    if (n > 0) hipLaunchKernelGGL(k_iota, dim3(grid_cap(n)), dim3(kBlock), 0, s, p, n);
}

void launch_sample_pivot(int in_mode, const View& g, uint64_t base, int sample, float q,
                         const float* mlp, float comps, int depth, Ctrl* ctrl, hipStream_t s) {
    if (in_mode == kOrig)
        hipLaunchKernelGGL(k_sample_pivot<kOrig>, dim3(1), dim3(kSampleThreads), 0, s, g, base,
                           sample, q, mlp, comps, depth, ctrl);
    else
        hipLaunchKernelGGL(k_sample_pivot<kCompact>, dim3(1), dim3(kSampleThreads), 0, s, g,
                           base, sample, q, mlp, comps, depth, ctrl);
}

void launch_split_count(int in_mode, const View& g, const uint64_t* pivot_dev, uint64_t* cnt,
                        uint64_t* bsum, Ctrl* ctrl, hipStream_t s) {
    if (g.len <= 0) return;
    const uint32_t nt = (uint32_t)((g.len + kRelabelTile - 1) / kRelabelTile);
    const unsigned per = kBlock / kWave;                   // tiles per workgroup step
    const unsigned grid = (nt + per - 1) / per < 4096u ? (nt + per - 1) / per : 4096u;
    const bool vec = ((((uintptr_t)g.w) | (in_mode == kOrig ? 0 : (uintptr_t)g.id)) & 15) == 0;
    if (in_mode == kOrig) {
        if (vec)
            hipLaunchKernelGGL((k_count_tiles<kOrig, true>), dim3(grid), dim3(kBlock), 0, s, g,
                               pivot_dev, cnt, nt);
        else
            hipLaunchKernelGGL((k_count_tiles<kOrig, false>), dim3(grid), dim3(kBlock), 0, s, g,
                               pivot_dev, cnt, nt);
    } else {
        if (vec)
            hipLaunchKernelGGL((k_count_tiles<kCompact, true>), dim3(grid), dim3(kBlock), 0, s,
                               g, pivot_dev, cnt, nt);
        else
            hipLaunchKernelGGL((k_count_tiles<kCompact, false>), dim3(grid), dim3(kBlock), 0, s,
                               g, pivot_dev, cnt, nt);
    }
    launch_scan_tiles(cnt, nt, bsum, &ctrl->light, s);
}

void launch_split(int in_mode, const View& g, int64_t n, const uint64_t* pivot_dev, EdgeSoA out,
                  const uint64_t* tile_off, Ctrl* ctrl, hipStream_t s) {
    if (g.len <= 0) return;
    const uint32_t nt = (uint32_t)((g.len + kRelabelTile - 1) / kRelabelTile);
    const unsigned grid = nt;             // one workgroup per tile measured fastest here
    if (in_mode == kOrig)
        hipLaunchKernelGGL((k_split<kOrig, true>), dim3(grid), dim3(kBlock), 0, s, g, n,
                           pivot_dev, out, tile_off, ctrl, nt);
    else
        hipLaunchKernelGGL((k_split<kCompact, false>), dim3(grid), dim3(kBlock), 0, s, g, n,
                           pivot_dev, out, tile_off, ctrl, nt);
}

void launch_rep_codes(const int32_t* P, int64_t n, uint64_t* codes, Ctrl* ctrl, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_giant_pick, dim3(1), dim3(kGiantThreads), 0, s, P, n, ctrl);
    const int64_t chunks = (n + 63) / 64;
    int64_t blocks = (chunks + kBlock / kWave - 1) / (kBlock / kWave);
    blocks = blocks > 4096 ? 4096 : blocks;
    hipLaunchKernelGGL(k_rep_codes, dim3((unsigned)blocks), dim3(kBlock), 0, s, P, n, ctrl, codes);
}

// orig: g is the caller's arrays and its heavy edges are those above `pivot`.
void launch_filter(const View& g, bool orig, uint64_t pivot, const int32_t* P,
                   const uint64_t* codes, const Ctrl* ctrl, uint64_t* flags, uint64_t* cnt,
                   uint64_t* bsum, EdgeSoA out, uint64_t* kept, hipStream_t s) {
    if (g.len <= 0) return;
    const uint32_t nt = (uint32_t)((g.len + kRelabelTile - 1) / kRelabelTile);
    const unsigned grid = nt < kTileGrid ? nt : kTileGrid;
    if (orig)
        hipLaunchKernelGGL(k_filter_flags<true>, dim3(grid), dim3(kBlock), 0, s, g, P, codes,
                           ctrl, pivot, flags, cnt, nt);
    else
        hipLaunchKernelGGL(k_filter_flags<false>, dim3(grid), dim3(kBlock), 0, s, g, P, codes,
                           ctrl, pivot, flags, cnt, nt);
    launch_scan_tiles(cnt, nt, bsum, kept, s);
    if (orig)
        hipLaunchKernelGGL(k_filter_scatter<true>, dim3(grid), dim3(kBlock), 0, s, g, P, codes,
                           ctrl, flags, cnt, out, nt);
    else
        hipLaunchKernelGGL(k_filter_scatter<false>, dim3(grid), dim3(kBlock), 0, s, g, P, codes,
                           ctrl, flags, cnt, out, nt);
}

// ------------------------------------------------------------------ driver

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Two edge buffers X, Y of m + 4 edges each.  A graph being split lives at
// [0, len) of one buffer (or in the caller's arrays at the top level); its
// split [light | heavy] goes to [0, len) of the other buffer.  Down the light
// recursion the lengths only shrink, so a split never reaches the heavy part
// an ancestor left at offset >= its light count; the filtered heavy edges are
// compacted leftwards to [0, kept) of their buffer before recursing on them.
size_t buffer_bytes(int64_t m) { return 4 * align_up((size_t)((m > 0 ? m : 1) + 4) * 4); }

EdgeSoA carve_buffer(char* p, int64_t m) {
    const size_t one = align_up((size_t)((m > 0 ? m : 1) + 4) * 4);
    EdgeSoA e;
    e.u = (int32_t*)p;
    e.v = (int32_t*)(p + one);
    e.w = (uint32_t*)(p + 2 * one);
    e.id = (uint32_t*)(p + 3 * one);
    return e;
}

struct Ctx {
    EngineBuffers B;
    EdgeSoA buf[2];
    int32_t* P;
    int64_t n;
    uint8_t* mask;
    hipStream_t s;
    msf_options opt;
    msf_stats* st;
    uint32_t splits;
    int sample;
    int64_t min_split;
    int sparse_deg;
    float q_net;   // quantile the network chose at the top split (0 = not yet)
    uint64_t* codes;   // 2-bit representative codes of the vertices
    uint64_t* flags;   // keep flags of the heavy edges being filtered
    uint64_t* bsum;    // chunk sums of the tile-count scans
    bool filtered;     // a filter step has run (ctrl->giant is meaningful)
    int retries;       // balanced-split retry: redraws per split (0 = off)
    int64_t defer;     // filtered sets below this size go back one level (0 = off)
};

View view_of(const EdgeSoA& e, int64_t len) {
    View g;
    g.u = e.u; g.v = e.v; g.w = e.w; g.id = e.id; g.p16 = nullptr; g.len = len;
    return g;
}

int compress_p(Ctx& C) {
    Ctrl* hc = host_ctrl();
    for (int attempt = 0;; ++attempt) {
        launch_zero_bytes((uint8_t*)&C.B.ctrl->jump_more, sizeof(uint32_t), C.s);
        const int h = prof_begin(K_PMAINT, C.s);
        launch_jump(C.P, C.n, 32, C.B.ctrl, C.s);
        prof_end(h, C.s, 12.0 * C.n);
        HIP_TRY(hipGetLastError());
        int st = read_ctrl(C.B.ctrl, hc, C.s);
        if (st) return st;
        if (!hc->jump_more) return MSF_OK;
        if (attempt > 64) {
            set_err_text("representative compression did not converge");
            return MSF_EINTERNAL;
        }
    }
}

int base_case(Ctx& C, int mode, const View& g) {
    C.st->base_cases += 1;
    // after a filter step the largest component's representative sits on most
    // of the surviving edges
    const int32_t hot = C.filtered ? host_ctrl()->giant : -1;
    return engine_solve(C.B, mode, g, C.n, C.mask, C.P, C.s, C.st, hot);
}

// The balanced-split retry's acceptance band (proof of the paper's Thm. 1:
// both sides in [|E|/3, 2|E|/3] for the median): the light fraction within 1/6
// of the target quantile.
bool balanced_split(int64_t light, int64_t total, float q) {
    const double qq = (double)q, l6 = 6.0 * (double)light;   // exact for the median
    return (6.0 * qq - 1.0) * (double)total <= l6 && l6 <= (6.0 * qq + 1.0) * (double)total;
}

// `where`: 0 / 1 = the graph lives at [0, len) of buffer X / Y, 2 = the
// caller's arrays.  *left = edges this call hands back to its caller (the
// deferral of small filtered sets, Sec. VI-C); they sit at [0, *left) of
// buffer X when where == 0, else of buffer Y.
int rec_filter(Ctx& C, int mode, const View& g, int where, int depth, int64_t* left) {
    *left = 0;
    if (g.len == 0) return MSF_OK;
    Ctrl* hc = host_ctrl();
    int st = read_ctrl(C.B.ctrl, hc, C.s);
    if (st) return st;
    // isSparse: average degree of the current components, or too few edges
    const double comps = (double)C.n - (double)hc->msf_edges;
    const bool sparse = g.len < C.min_split || 2.0 * (double)g.len <= C.sparse_deg * comps ||
                        depth >= kMaxDepth;
    if (sparse) return base_case(C, mode, g);

    const uint32_t split = C.splits++;
    // The network picks one quantile per call, on the top split's sample;
    // deeper splits reuse it (a constant quantile per call is also what its
    // training targets were measured with).
    float q = C.opt.pivot == MSF_PIVOT_QUANTILE ? C.opt.quantile : 0.5f;
    const float* net = nullptr;
    if (C.opt.pivot == MSF_PIVOT_MLP) {
        if (C.q_net > 0.f) q = C.q_net;
        else net = mlp_device_params();
    }
    const int tgt = where == 0 ? 1 : 0;
    const EdgeSoA R = C.buf[tgt];
    uint32_t attempt = 0;
    int h;
    for (;; ++attempt) {
        h = prof_begin(K_SAMPLE, C.s);
        launch_sample_pivot(mode, g, pivot_stream_base(C.opt.seed, split, attempt), C.sample, q,
                            net, (float)comps, depth, C.B.ctrl, C.s);
        prof_end(h, C.s, 8.0 * C.sample);
        h = prof_begin(K_PARTITION, C.s);
        launch_split_count(mode, g, &C.B.ctrl->pivot, C.B.status, C.bsum, C.B.ctrl, C.s);
        prof_end(h, C.s, (mode == kOrig ? 4.0 : 8.0) * g.len);
        if (attempt >= (uint32_t)C.retries) break;
        // the retry: is the split balanced?  (one more host read per draw)
        HIP_TRY(hipGetLastError());
        if ((st = read_ctrl(C.B.ctrl, hc, C.s))) return st;
        if (net) {                  // later draws reuse the network's quantile
            q = hc->q_used;
            net = nullptr;
        }
        if (balanced_split((int64_t)hc->light, g.len, hc->q_used)) break;
        C.st->pivot_retries += 1;
    }
    h = prof_begin(K_PARTITION, C.s);
    launch_split(mode, g, C.n, &C.B.ctrl->pivot, R, C.B.status, C.B.ctrl, C.s);
    // split reads (12 B per edge on the caller's arrays, 16 B on a buffer) and
    // writes: everything on a buffer, the light part only on top
    prof_end(h, C.s, mode == kOrig ? 12.0 * g.len : 32.0 * g.len);
    HIP_TRY(hipGetLastError());
    if ((st = read_ctrl(C.B.ctrl, hc, C.s))) return st;
    if (hc->err & kErrRange) return MSF_ERANGE;
    if (hc->err) {
        set_err_text("device error bits during a split");
        return MSF_EINTERNAL;
    }
    const int64_t nl = (int64_t)hc->light, nh = g.len - nl;
    if (mode == kOrig) prof_add(K_PARTITION, 16.0 * nl);
    if (split < MSF_MAX_TRACE) {
        C.st->split_edges[split] = (uint64_t)g.len;
        C.st->split_pivot[split] = hc->pivot;
        C.st->split_light[split] = (uint64_t)nl;
        C.st->split_q[split] = hc->q_used;
        C.st->split_kept[split] = 0;
        C.st->split_attempts[split] = attempt + 1;
        memcpy(C.st->split_features[split], hc->feat, sizeof C.st->split_features[split]);
    }
    if (split == 0) {
        C.q_net = hc->q_used;
        C.st->pivot_q_used = hc->q_used;
        memcpy(C.st->top_features, hc->feat, sizeof C.st->top_features);
    }
    C.st->levels += 1;
    if (nl == 0 || nh == 0) return base_case(C, mode, g);   // degenerate pivot

    // Heavy part: right after the light part in R, or (top level) the
    // caller's arrays themselves, where the split wrote nothing heavy.
    const bool heavy_in_place = mode == kOrig;
    const uint64_t pivot = hc->pivot;
    View Hv;
    if (heavy_in_place) {
        Hv = g;
    } else {
        EdgeSoA H = R;
        const int64_t nl_al = (nl + 3) & ~(int64_t)3;
        H.u += nl_al; H.v += nl_al; H.w += nl_al; H.id += nl_al;
        Hv = view_of(H, nh);
    }
    // The light recursion; the edges it hands back (at [0, nd) of R, below
    // this graph's heavy part) are filtered first, together with the heavy part.
    int64_t nd = 0;
    if ((st = rec_filter(C, kCompact, view_of(R, nl), tgt, depth + 1, &nd))) return st;

    // Filter: drop heavy edges inside a light component; the rest, relabelled
    // and in order, go to [0, kept) of the other buffer, which holds nothing
    // live below this graph's length (this graph itself is no longer needed):
    // the handed-back edges first (their keys lie below the heavy ones, so
    // positions still order equal weights by id), then the heavy ones.
    if ((st = compress_p(C))) return st;
    h = prof_begin(K_PMAINT, C.s);
    launch_rep_codes(C.P, C.n, C.codes, C.B.ctrl, C.s);
    C.filtered = true;
    prof_end(h, C.s, 4.0 * C.n + C.n / 4.0);
    const int o = 1 - tgt;
    int64_t kd = 0;
    if (nd > 0) {
        h = prof_begin(K_FILTER, C.s);
        launch_filter(view_of(R, nd), false, pivot, C.P, C.codes, C.B.ctrl, C.flags, C.B.status,
                      C.bsum, C.buf[o], &C.B.ctrl->m_next, C.s);
        prof_end(h, C.s, 8.0 * nd);
        HIP_TRY(hipGetLastError());
        if ((st = read_ctrl(C.B.ctrl, hc, C.s))) return st;
        kd = (int64_t)hc->m_next;
        prof_add(K_FILTER, 24.0 * kd);
    }
    EdgeSoA out = C.buf[o];
    out.u += kd; out.v += kd; out.w += kd; out.id += kd;
    h = prof_begin(K_FILTER, C.s);
    launch_filter(Hv, heavy_in_place, pivot, C.P, C.codes, C.B.ctrl, C.flags, C.B.status,
                  C.bsum, out, &C.B.ctrl->m_next, C.s);
    prof_end(h, C.s, heavy_in_place ? 12.0 * g.len : 8.0 * nh);
    HIP_TRY(hipGetLastError());
    if ((st = read_ctrl(C.B.ctrl, hc, C.s))) return st;
    int64_t kept = kd + (int64_t)hc->m_next;
    prof_add(K_FILTER, 24.0 * (kept - kd));
    C.st->filtered_in += (uint64_t)(nh + nd);
    C.st->filtered_out += (uint64_t)kept;
    if (split < MSF_MAX_TRACE) {
        C.st->split_kept[split] = (uint64_t)kept;
        C.st->split_deferred_in[split] = (uint64_t)nd;
    }
    // The filtered edges sit at [0, kept) of buffer o; a recursion on them
    // (where = o) hands its leftovers back at [0, left) of the same buffer.
    while (kept > 0) {
        if (depth > 0 && kept < C.defer) {      // too few: merge them one level up
            C.st->deferrals += 1;
            *left = kept;
            return MSF_OK;
        }
        int64_t back = 0;
        if ((st = rec_filter(C, kCompact, view_of(C.buf[o], kept), o, depth + 1, &back)))
            return st;
        kept = back;
    }
    return MSF_OK;
}

}  // namespace

size_t codes_bytes(int64_t n) { return align_up(((size_t)((n > 0 ? n : 1) + 63) / 64) * 16); }
size_t flags_bytes(int64_t m) {
    return align_up(((size_t)((m > 0 ? m : 1) + kRelabelTile - 1) / kRelabelTile) *
                    (kRelabelTile / 64) * 8);
}

size_t filter_bytes(int64_t m, int64_t n, const msf_options& opt) {
    return engine_bytes(m, n, opt.round0 != MSF_ROUND0_EDGES,
                        opt.dedup_policy == MSF_DEDUP_EXACT) + align_up((size_t)(n > 0 ? n : 1) * 4) + 2 * buffer_bytes(m) +
           codes_bytes(n) + flags_bytes(m) + align_up(kScanTop * 8);
}

int filter_solve(const int32_t* u, const int32_t* v, const uint32_t* w, int64_t m, int64_t n,
                 uint8_t* mask, char* ws, hipStream_t s, const msf_options& opt,
                 msf_stats* stats) {
    Ctx C;
    size_t off = engine_carve(ws, m, n, &C.B, opt.round0 != MSF_ROUND0_EDGES,
                              opt.dedup_policy == MSF_DEDUP_EXACT);
    C.B.round0 = opt.round0;
    C.B.dedup = opt.dedup_policy;
    C.B.tail = opt.tail_threshold;
    C.P = (int32_t*)(ws + off);
    off += align_up((size_t)(n > 0 ? n : 1) * 4);
    C.buf[0] = carve_buffer(ws + off, m);
    C.buf[1] = carve_buffer(ws + off + buffer_bytes(m), m);
    off += 2 * buffer_bytes(m);
    C.codes = (uint64_t*)(ws + off);
    off += codes_bytes(n);
    C.flags = (uint64_t*)(ws + off);
    off += flags_bytes(m);
    C.bsum = (uint64_t*)(ws + off);
    C.n = n;
    C.mask = mask;
    C.s = s;
    C.opt = opt;
    C.st = stats;
    C.splits = 0;
    C.q_net = 0.f;
    C.filtered = false;
    C.sample = opt.sample_size > 0 ? opt.sample_size : 4096;
    C.min_split = opt.min_split_edges > 0 ? opt.min_split_edges : (1 << 20);
    C.sparse_deg = opt.sparse_degree > 0 ? opt.sparse_degree : 4;
    C.retries = opt.split_retries;
    C.defer = opt.defer_edges;

    launch_zero_bytes((uint8_t*)C.B.ctrl, sizeof(Ctrl), s);
    int h = prof_begin(K_FILL, s);
    launch_zero_bytes(mask, m, s);
    launch_iota(C.P, n, s);
    prof_end(h, s, (double)m + 4.0 * n);
    View g{u, v, nullptr, w, nullptr, m};
    int64_t left = 0;
    int st = rec_filter(C, kOrig, g, 2, 0, &left);
    if (st) return st;
    if (left != 0) {
        set_err_text("the top level of Filter-Boruvka handed edges back");
        return MSF_EINTERNAL;
    }
    Ctrl* hc = host_ctrl();
    if ((st = read_ctrl(C.B.ctrl, hc, s))) return st;
    stats->total_weight = hc->total;
    stats->msf_edges = hc->msf_edges;
    return MSF_OK;
}

}  // namespace msf
