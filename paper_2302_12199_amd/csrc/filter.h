// Filter-Borůvka driver (paper Sec. V, Alg. 2) on one GPU.
#pragma once
#include "engine.h"

namespace msf {

size_t filter_bytes(int64_t m, int64_t n, const msf_options& opt);
int filter_solve(const int32_t* u, const int32_t* v, const uint32_t* w, int64_t m, int64_t n,
                 uint8_t* mask, char* ws, hipStream_t s, const msf_options& opt,
                 msf_stats* stats);

// Stream base of the pivot sampler for split number `split` (depth-first
// order): SplitMix64 output function applied as mix(mix(seed) ^ (tag + split)).
uint64_t pivot_stream_base(uint64_t seed, uint32_t split, uint32_t attempt);

// filter.hip launchers
void launch_sample_pivot(int in_mode, const View& g, uint64_t base, int sample, float q,
                         const float* mlp, float comps, int depth, Ctrl* ctrl, hipStream_t s);
void launch_split_count(int in_mode, const View& g, const uint64_t* pivot_dev, uint64_t* cnt,
                        uint64_t* bsum, Ctrl* ctrl, hipStream_t s);
void launch_split(int in_mode, const View& g, int64_t n, const uint64_t* pivot_dev, EdgeSoA out,
                  const uint64_t* tile_off, Ctrl* ctrl, hipStream_t s);
void launch_iota(int32_t* p, int64_t n, hipStream_t s);

}  // namespace msf
