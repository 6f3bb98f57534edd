// Round 0 by vertex buckets: the lightest-edge search and the relabelling
// pass of the first Borůvka round (paper Sec. II-C) without random accesses
// into n-sized tables.
#pragma once
#include "common.h"

namespace msf {

constexpr int kBucketShift = 14;                      // 2^14 vertices per bucket
constexpr int64_t kBucketWidth = 1ll << kBucketShift;
constexpr int kBucketTileShift = 13;
constexpr int64_t kBucketTile = 1ll << kBucketTileShift;   // edges per tile
constexpr int64_t kTileArcs = 2 * kBucketTile;              // arc slots per tile block
constexpr int kBucketMax = 1024;                      // buckets (n <= 2^24)
constexpr int kArcSideBit = kBucketShift + kBucketTileShift;   // which end of its edge an arc is
constexpr int kBucketThreads = 1024;

struct BucketBuffers {
    uint64_t* arcs;      // [nt * kTileArcs] per tile, its arcs sorted by bucket:
                         // w << 32 | side << 27 | (edge - first edge of the tile) << 14 |
                         // vertex in bucket (side 1: the edge's v end); later the arcs'
                         // new labels, bucket-major (uint32)
    uint32_t* meta;      // [nt * nb] tile-major: run start in the tile block | run length << 16
    uint32_t* metat;     // [nb * nt] the same, bucket-major
    uint32_t* offb;      // [nb * nt] bucket-major: first arc of run (b, t) counted from the bucket's start
    uint32_t* offt;      // [nt * nb] the same, tile-major
    uint64_t* base;      // [nb + 1] first arc of each bucket in the bucket-major streams
    uint64_t* tmp;       // scan partial sums
    uint16_t* xs;        // [2m] bucket-major: vertex in bucket of every arc
    uint32_t* rank;      // [m] places of the edge's two arcs in its tile block (u | v << 16);
                         // 0 for an edge without arcs (self-loop, id out of range)
    uint64_t* hotpre;    // [n + 2] sample counts of the round-1 labels, tier flags, their
                         // exclusive scan (hotpre[hotn] = tier sizes), labels sampled
    uint64_t* hottmp;    // scan partial sums
    mutable int64_t hotn;  // labels of the last hot-first renumbering (hotpre[hotn + 1] = sampled)
    int64_t mcap, ncap;  // the largest graph the buffers were carved for
};

// Graphs the bucketed round 0 is sized for (the workspace holds its buffers).
bool bucket_eligible(int64_t m, int64_t n);
size_t bucket_carve(char* ws, int64_t m, int64_t n, BucketBuffers* B);   // bytes (0 if not eligible)
// The buffers were carved and fit a graph of m edges and n vertices.
bool bucket_usable(const BucketBuffers& B, int64_t m, int64_t n);

// ctrl->aux[0] = edges among kLocalitySample, sampled evenly, whose ends are
// less than a bucket width apart (m >= kLocalitySample).
constexpr int kLocalitySample = 4096;
void bucket_sample_locality(const int32_t* u, const int32_t* v, int64_t m, Ctrl* ctrl,
                            hipStream_t s);

// Lightest edge of every vertex: best[0, n) (validates the ids: kErrRange),
// as w << 32 | position << 1 | side, side 1 when the vertex is the edge's v
// end (the bucketed path takes m < 2^31, so this fits; the order is that of
// (w, position): only a self-loop has both ends at one vertex, and it has no
// arcs).  The hook then reads one end of the edge, not both.
void bucket_minedge(const BucketBuffers& B, const int32_t* u, const int32_t* v,
                    const uint32_t* w, int64_t m, int64_t n, uint64_t* best, Ctrl* ctrl,
                    hipStream_t s);
// Renumbers the round-1 labels lab[0, nr) (values in [0, nn), -1 = none) so
// that the labels on many sampled edge ends come first.
void bucket_hot_first(const BucketBuffers& B, const int32_t* u, const int32_t* v, int64_t m,
                      int32_t* lab, int64_t nr, int64_t nn, hipStream_t s);

// Relabel every edge through M (round-0 vertex -> next label), write the
// OUT layout (kOut32 or kOut16; dead edges as (0, 0)), count the live edges
// into ctrl->m_next and run the next round's lightest-edge search into
// best_next[0, nn), as side keys (w << 32 | position << 1 | side, side 1 at
// the edge's v end).  Uses the arcs of the last bucket_minedge call on the
// same edges.
void bucket_relabel(const BucketBuffers& B, const uint32_t* w, int64_t m, int64_t n,
                    const int32_t* M, int out,
                    int32_t* ou, int32_t* ov, uint32_t* op16, uint64_t* best_next, int64_t nn,
                    Ctrl* ctrl, hipStream_t s);

}  // namespace msf
