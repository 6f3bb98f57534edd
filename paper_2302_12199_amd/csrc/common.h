// Shared device/host definitions of the MSF library (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace msf {

constexpr int kBlock = 256;                 // threads per workgroup (4 waves)
constexpr int kWave = 64;                   // CDNA wavefront width
constexpr int kItems = 16;                  // items per thread in scan tiles
constexpr int kTile = kBlock * kItems;      // items per decoupled-lookback tile
constexpr int kRelabelItems = 8;            // edges per thread in the relabel pass
constexpr int kRelabelTile = kBlock * kRelabelItems;
constexpr int kPassBlock = 1024;            // threads per streaming-pass workgroup
constexpr int kPassGroups = 2;              // 4-edge groups per lane per step in a pass
constexpr uint64_t kKeyMax = ~0ull;         // "no edge" in best[]

// Error bits accumulated on the device.
constexpr uint32_t kErrRange = 1u;          // an endpoint id outside [0, n)
constexpr uint32_t kErrLookback = 2u;       // a lookback wait hit its spin bound
constexpr uint32_t kErrInternal = 4u;       // a min edge not incident to its vertex

// Device control block (lives in the workspace; zeroed per call).
struct Ctrl {
    uint32_t tile_counter;   // dynamic tile ids of the running lookback scan
    uint32_t err;            // kErr* bits
    uint32_t jump_more;      // pointer jumping has not reached a fixed point yet
    uint32_t pad0;
    uint64_t n_next;         // vertices of the next round (root scan result)
    uint64_t m_next;         // edges of the next round (edge compaction result)
    uint64_t total;          // MSF weight so far
    uint64_t msf_edges;      // MSF edges so far
    uint64_t live;           // vertices with an incident edge, this round
    uint64_t found;          // MSF edges marked this round
    uint64_t light;          // filter: edges with key <= pivot
    uint64_t pivot;          // filter: pivot key of the current split
    float q_used;            // filter: sample quantile used
    int32_t giant;           // filter: representative of the largest sampled component (-1: none)
    uint32_t tail_rounds;    // rounds run by the single-workgroup tail
    uint32_t tail_edges;     // distinct vertex pairs handed to the tail
    uint32_t tail_live[24];  // per tail round: vertices with an incident edge
    uint32_t tail_found[24]; // per tail round: MSF edges found
    uint32_t tail_scan[24];  // per tail round: live pairs scanned
    float feat[16];          // filter: features of the last pivot sample
    uint64_t aux[4];         // spare
};

constexpr int kTailMax = 1024;              // vertices the single-workgroup tail handles
constexpr int64_t kTailAutoPairs = 65536;   // automatic hand-over: at most this many pairs
constexpr int kTailThreads = 1024;
constexpr int kTailRoundsMax = 24;
// Labels whose vertex pairs the pass before the tail keeps in LDS (128 * 127 / 2
// slots, 63.5 KiB), after the labels of that round were renumbered hot first.
constexpr int64_t kPairHot = 128;

// Lookback status word: 2 flag bits over a 62-bit inclusive/aggregate value.
constexpr uint64_t kStatAgg = 1ull << 62;
constexpr uint64_t kStatInc = 2ull << 62;
constexpr uint64_t kStatMask = (1ull << 62) - 1;
constexpr uint32_t kSpinLimit = 1u << 24;

// Edge arrays of a round: structure of arrays, 16 B per edge.  Position order
// equals edge-id order (every compaction is stable), so inside a round the key
// (w << 32 | position) orders edges exactly like (w, id).
struct EdgeSoA {
    int32_t* u;
    int32_t* v;
    uint32_t* w;
    uint32_t* id;
};

// How the edges of the current graph are stored.  In every layout the
// position of an edge is increasing in its id, so (w << 32 | position) is a
// key with the paper's tie break.
//   kOrig     the caller's arrays: u, v, w; id = position
//   kFull32   int32 endpoint labels for every input edge (dead edges hold an
//             equal pair); w = caller's w; id = position
//   kFull16   both endpoint labels packed into one uint32 (a | b << 16) for
//             every input edge, usable once labels fit in 16 bits
//   kCompact  only live edges, stably compacted: u, v, w, id arrays
enum ViewMode { kOrig = 0, kFull32 = 1, kFull16 = 2, kCompact = 3 };

struct View {
    const int32_t* u;
    const int32_t* v;
    const uint32_t* p16;
    const uint32_t* w;
    const uint32_t* id;
    int64_t len;        // positions in the arrays
};

// Outputs of a streaming pass.
enum PassOut { kOutNone = 0, kOut32 = 1, kOut16 = 2 };

// Parallel-edge removal in a compaction: none, per tile (an LDS hash table),
// or exact (a global hash table filled by a pass before the compaction).
enum DedupKind { kDedupNone = 0, kDedupLocal = 1, kDedupExact = 2 };

}  // namespace msf
