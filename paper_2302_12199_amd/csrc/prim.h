// Wave and workgroup primitives for gfx950 (wave64): ballot-based stream
// compaction ranks, wave reductions and a decoupled-lookback tile prefix.
#pragma once
#include "common.h"

namespace msf {

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// Workgroups are handed to the XCDs in turn (id mod kXcds), each XCD with its
// own L2.  xcd_slot renumbers the ids 0..G-1 so that the workgroups of one XCD
// take consecutive slots: neighbouring tiles or buckets, which share the cache
// lines at their boundaries, are then read through the same L2.  A bijection
// on [0, G) whatever the real XCD count.
constexpr uint32_t kXcds = 8;
__device__ __forceinline__ uint32_t xcd_slot(uint32_t i, uint32_t G) {
    const uint32_t x = i % kXcds, r = i / kXcds;
    return x * (G / kXcds) + (x < G % kXcds ? x : G % kXcds) + r;
}

// Number of set bits of `mask` in lanes below the calling lane.
__device__ __forceinline__ uint32_t lanes_below(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t x) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    return x;
}

__device__ __forceinline__ uint64_t ld_relaxed(const uint64_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_relaxed(uint64_t* p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// min-update of a 64-bit packed key: read first, issue the atomic only when it
// can still lower the value.  Stale reads are harmless: best[] only decreases.
__device__ __forceinline__ void atomic_min_key(uint64_t* p, uint64_t key) {
    if (key < *p) atomicMin((unsigned long long*)p, (unsigned long long)key);
}

__device__ __forceinline__ uint64_t wave_min_u64(uint64_t x) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const uint64_t y = __shfl_xor(x, off, 64);
        x = y < x ? y : x;
    }
    return x;
}

// atomic_min_key(&best[t], key) for every lane with `act`, called by the
// whole wave.  Lanes aiming at the same entry as the first active lane are
// first min-reduced across the wave and update it once: edges of one hot
// component would otherwise queue on a single address.
__device__ __forceinline__ void wave_min_update(uint64_t* best, int32_t t, uint64_t key,
                                                bool act) {
    const uint64_t am = __ballot(act);
    if (am == 0) return;
    const int leader = __builtin_ctzll(am);
    const int32_t tl = __shfl(t, leader, 64);
    const bool same = act && t == tl;
    if (__popcll(__ballot(same)) > 1) {
        const uint64_t k = wave_min_u64(same ? key : kKeyMax);
        if (lane_id() == leader) atomic_min_key(&best[tl], k);
        act = act && !same;
    }
    if (act) atomic_min_key(&best[t], key);
}

// As wave_min_update, for lanes whose key already beat the entry's value as
// read earlier (a caller that issues all its reads first keeps them in
// flight together): the atomics go out without reading the entry again.
__device__ __forceinline__ void wave_min_commit(uint64_t* best, int32_t t, uint64_t key,
                                                bool act) {
    const uint64_t am = __ballot(act);
    if (am == 0) return;
    const int leader = __builtin_ctzll(am);
    const int32_t tl = __shfl(t, leader, 64);
    const bool same = act && t == tl;
    if (__popcll(__ballot(same)) > 1) {
        const uint64_t k = wave_min_u64(same ? key : kKeyMax);
        if (lane_id() == leader) atomicMin((unsigned long long*)&best[tl], (unsigned long long)k);
        act = act && !same;
    }
    if (act) atomicMin((unsigned long long*)&best[t], (unsigned long long)key);
}

// Hot labels of a workgroup: called by one wave with one sampled label per
// lane (-1 = none); writes the kHot most frequent sampled labels that occur
// at least kHotMinCount times (else -1) and clears their minima.
constexpr int kHot = 4;
constexpr int kHotMinCount = 4;
__device__ __forceinline__ void hot_labels(int32_t lab, int32_t* s_hot,
                                           unsigned long long* s_hotmin) {
    for (int h = 0; h < kHot; ++h) {
        int best_cnt = 0;
        int32_t best_lab = -1;
        for (int i = 0; i < kWave; ++i) {
            const int32_t li = __shfl(lab, i, kWave);
            const int c = __popcll(__ballot(lab == li && li >= 0));
            if (c > best_cnt) { best_cnt = c; best_lab = li; }
        }
        if (lane_id() == 0) {
            s_hot[h] = best_cnt >= kHotMinCount ? best_lab : -1;
            s_hotmin[h] = kKeyMax;
        }
        if (best_lab >= 0 && lab == best_lab) lab = -1;   // next pass finds the next label
    }
}
// If t is one of the hot labels, min-updates its LDS entry and returns true.
__device__ __forceinline__ bool hot_min(const int32_t (&hot)[kHot], unsigned long long* s_hotmin,
                                        int32_t t, uint64_t key) {
#pragma unroll
    for (int h = 0; h < kHot; ++h) {
        if (t == hot[h]) {
            if (key < s_hotmin[h]) atomicMin(&s_hotmin[h], (unsigned long long)key);
            return true;
        }
    }
    return false;
}

// Dynamic tile id: tiles are numbered in the order workgroups start, so a tile
// only ever waits on tiles that are already running (no deadlock).
__device__ __forceinline__ uint32_t take_tile(Ctrl* ctrl, uint32_t* s_tile) {
    if (threadIdx.x == 0) *s_tile = atomicAdd(&ctrl->tile_counter, 1u);
    __syncthreads();
    return *s_tile;
}

// Exclusive prefix of this tile's aggregate over all earlier tiles
// (single-pass scan with decoupled lookback).  Must be called by the whole
// workgroup; wave 0 does the lookback, 64 predecessors per step.  Every wait
// is bounded: past kSpinLimit polls the error bit is raised and the missing
// value is taken as zero, so the kernel always terminates.
__device__ __forceinline__ uint64_t tile_prefix(uint64_t* status, uint32_t tile, uint64_t agg,
                                                Ctrl* ctrl, uint64_t* s_prefix) {
    if (threadIdx.x < kWave) {
        const int lane = threadIdx.x;
        uint64_t excl = 0;
        if (tile == 0) {
            if (lane == 0) st_relaxed(&status[0], kStatInc | agg);
        } else {
            if (lane == 0) st_relaxed(&status[tile], kStatAgg | agg);
            int64_t base = (int64_t)tile - 1;
            while (true) {
                const int64_t idx = base - lane;
                uint64_t s = kStatInc;  // before tile 0: inclusive zero
                uint32_t spins = 0;
                while (true) {
                    if (idx >= 0) s = ld_relaxed(&status[idx]);
                    const uint64_t pending = __ballot((s >> 62) == 0);
                    if (pending == 0) break;
                    if (++spins > kSpinLimit) {
                        if (lane == 0) atomicOr(&ctrl->err, kErrLookback);
                        if ((s >> 62) == 0) s = kStatInc;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                }
                const uint64_t inc = __ballot((s >> 62) == 2);
                if (inc) {
                    const int first = __builtin_ctzll(inc);  // closest inclusive predecessor
                    excl += wave_sum_u64(lane <= first ? (s & kStatMask) : 0);
                    break;
                }
                excl += wave_sum_u64(s & kStatMask);
                base -= kWave;
            }
            if (lane == 0) st_relaxed(&status[tile], kStatInc | (excl + agg));
        }
        if (lane == 0) *s_prefix = excl;
    }
    __syncthreads();
    return *s_prefix;
}

// Exclusive scan of one value per thread over the workgroup; *total gets the
// sum.  Every thread of the workgroup must call it (two barriers inside).
__device__ __forceinline__ uint64_t block_excl_scan(uint64_t x, uint64_t* s_w, uint64_t* total) {
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    uint64_t inc = x;
    for (int off = 1; off < kWave; off <<= 1) {
        const uint64_t y = __shfl_up(inc, off, kWave);
        if (lane >= off) inc += y;
    }
    if (lane == kWave - 1) s_w[wave] = inc;
    __syncthreads();
    uint64_t pre = 0, tot = 0;
    const int nw = blockDim.x / kWave;
    for (int i = 0; i < nw; ++i) {
        const uint64_t v = s_w[i];
        if (i < wave) pre += v;
        tot += v;
    }
    __syncthreads();
    *total = tot;
    return pre + inc - x;
}

// Stores 4 consecutive relabelled positions of a pass (q = position / 4) in
// the layout OUT selects: int32 label pairs or 16-bit packed pairs.
// NT: non-temporal stores, for output that leaves the L2 to reused tables.
template <int OUT, bool NT = false>
__device__ __forceinline__ void store_group(int64_t q, int64_t m, const int32_t (&ra)[4],
                                            const int32_t (&rb)[4], int32_t* __restrict__ ou,
                                            int32_t* __restrict__ ov,
                                            uint32_t* __restrict__ op16) {
    const int64_t e0 = q * 4;
    const bool full = e0 + 3 < m;
    if constexpr (OUT == kOut32) {
        if (full && NT) {
            typedef int32_t i32x4 __attribute__((ext_vector_type(4)));
            __builtin_nontemporal_store(i32x4{ra[0], ra[1], ra[2], ra[3]},
                                        reinterpret_cast<i32x4*>(ou) + q);
            __builtin_nontemporal_store(i32x4{rb[0], rb[1], rb[2], rb[3]},
                                        reinterpret_cast<i32x4*>(ov) + q);
        } else if (full) {
            reinterpret_cast<int4*>(ou)[q] = make_int4(ra[0], ra[1], ra[2], ra[3]);
            reinterpret_cast<int4*>(ov)[q] = make_int4(rb[0], rb[1], rb[2], rb[3]);
        } else {
            for (int k = 0; k < 4; ++k)
                if (e0 + k < m) { ou[e0 + k] = ra[k]; ov[e0 + k] = rb[k]; }
        }
    } else if constexpr (OUT == kOut16) {
        uint32_t pk[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) pk[k] = (uint32_t)ra[k] | ((uint32_t)rb[k] << 16);
        if (full && NT) {
            typedef uint32_t u32x4v __attribute__((ext_vector_type(4)));
            __builtin_nontemporal_store(u32x4v{pk[0], pk[1], pk[2], pk[3]},
                                        reinterpret_cast<u32x4v*>(op16) + q);
        } else if (full) {
            reinterpret_cast<uint4*>(op16)[q] = make_uint4(pk[0], pk[1], pk[2], pk[3]);
        } else {
            for (int k = 0; k < 4; ++k)
                if (e0 + k < m) op16[e0 + k] = pk[k];
        }
    }
}

}  // namespace msf
