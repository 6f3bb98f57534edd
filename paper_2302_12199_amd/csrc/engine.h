// Borůvka round driver (paper Sec. II-C, Alg. 1's round loop) on one GPU.
#pragma once
#include "bucket.h"
#include "host.h"
#include "launch.h"

namespace msf {

// Device buffers of the round loop, carved out of the caller's workspace.
struct EngineBuffers {
    Ctrl* ctrl;
    uint64_t* status;     // lookback tile status words; tile counts of a compaction
    uint64_t* cflags;     // compaction keep bits, one per position
    uint64_t* cbsum;      // compaction scan chunk sums
    uint64_t* best[2];    // lightest-edge keys, this round / next round
    int32_t* parent;
    uint64_t* rootbits;   // the hook's root and live bits, one word per 64 vertices
    uint64_t* livebits;
    int32_t* lab[2];      // per-round label arrays (alternating)
    int32_t* map[2];      // composed label maps (alternating)
    int32_t* orig[2];     // representative-tracking: input vertex of each round vertex
    int32_t* f32u;        // kFull32 layout
    int32_t* f32v;
    uint32_t* p16;        // kFull16 layout
    EdgeSoA cbuf[2];      // kCompact layouts (alternating)
    uint64_t* pairs;      // tail: lightest edge per vertex pair (triangular table)
    int32_t* perm;        // tail: hot-first permutation of its vertices' labels
    uint32_t* list_xy[2];  // tail: pair list (ping-pong, compacted every round)
    uint64_t* list_key[2];
    uint64_t* dpair;      // exact parallel-edge removal: global hash table, vertex pairs
    uint64_t* dmin;       //   and the lightest key of each (dslots entries each)
    int64_t dslots;       //   0 when the workspace holds no table
    BucketBuffers bk;     // bucketed round 0 (large graphs only)
    int round0;           // msf_round0: when round 0 runs by buckets
    int dedup;            // msf_dedup: parallel-edge removal in the compactions
    int64_t tail;         // the tail takes over at <= tail labels (1..kTailMax); 0 = automatic
    int64_t ncap, mcap;
};

// buckets: also carve the bucketed round 0's buffers (for graphs it applies to);
// exact: also carve the global pair table of exact parallel-edge removal.
size_t engine_bytes(int64_t m, int64_t n, bool buckets, bool exact);
// Carves buffers starting at ws; returns the bytes used.
size_t engine_carve(char* ws, int64_t m, int64_t n, EngineBuffers* B, bool buckets, bool exact);

// Runs Borůvka rounds until no edge is left.
//   view/mode   the current graph: kOrig (the caller's arrays; round 0 runs
//               the lightest-edge pass first) or kCompact (ids already set)
//   nv          vertex ids of the view are in [0, nv)
//   rep         optional int32[nv]: representative tracking for Filter-
//               Borůvka.  rep[x] = x on entry for the vertices in the view;
//               on return every vertex that was contracted points (directly
//               or through a chain) to the vertex it was merged into.
//   hot         a vertex of the view expected on very many edges, or -1
//               (its round-0 minimum is reduced per workgroup in LDS)
// Marks MSF edges in mask[] and accumulates total/msf_edges in B.ctrl.
int engine_solve(EngineBuffers& B, int mode, const View& view, int64_t nv, uint8_t* mask,
                 int32_t* rep, hipStream_t s, msf_stats* stats, int32_t hot = -1);

}  // namespace msf
