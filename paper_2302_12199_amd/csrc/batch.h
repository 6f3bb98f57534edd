// Batched solver: arguments shared by the kernel (batch.hip) and its C ABI
// (batch_api.hip).
#pragma once
#include "common.h"

namespace msf {

constexpr int kMaxXcd = 16;          // XCC_ID is a 4-bit field
constexpr int kCoopVertsPerThread = 8;
constexpr int kCoopEdgesPerThread = 16;
constexpr int kMinBatchBlock = 256;
constexpr int kCoopPairsPerThread = 16;
// Once a cooperative graph has at most kPairMax live vertices, its edges are
// reduced to the lightest edge per vertex pair (a triangular table) and the
// remaining rounds scan the table instead of the edges.
constexpr int64_t kPairMax = 4096;

// Per-launch counters at the start of the workspace (zeroed by k_batch_prep).
struct BatchQueue {
    uint32_t big_next;              // next index into the cooperative list
    uint32_t small_next;            // next index into the workgroup list
    uint32_t nbig;                  // graphs solved cooperatively
    uint32_t err;                   // a bounded wait ran out (results invalid)
    uint32_t tiny_next;             // next index into the wave list
    uint32_t ntiny;                 // graphs solved by one wave each
    uint32_t nsmall;                // graphs solved by one workgroup each
    uint32_t pad;
};

// Cooperative solve of one graph at a time by every workgroup of one XCD.
// Work is cut into phases of chunks; a workgroup takes a chunk with one
// atomic on `ticket` (phase << 32 | chunk), and the one that completes the
// last chunk of a phase sets up the next.  A workgroup waits only for chunks
// that running workgroups have taken, so no co-residency is assumed.
struct alignas(256) XcdWork {
    uint64_t ticket;                // phase << 32 | next chunk
    uint32_t done[2];               // completed chunks, by phase parity
    uint32_t kind[2];               // phase kind, by parity
    uint32_t nchunks[2];            // chunks of the phase, by parity
    uint32_t state;                 // 0 idle, 1 claimed by a workgroup
    uint32_t round;                 // Borůvka round of the current graph
    uint32_t jit;                   // pointer-jumping step
    uint32_t f_any, f_bad, f_changed;
    uint32_t pair_mode;             // rounds scan the pair table
    int64_t graph, n, m;            // current graph
    int64_t ncur, nnext;            // live vertices this round / next round
    int64_t pn;                     // vertices of the pair table
    uint64_t total;                 // MSF weight so far
};

struct BatchArgs {
    const int32_t* u;
    const int32_t* v;
    const uint32_t* w;
    const int64_t* eoff;     // [G + 1] edge offsets
    const int64_t* voff;     // [G + 1] vertex offsets
    int64_t G;
    const int32_t* order;    // [G] processing order, or null
    uint8_t* mask;           // [eoff[G]]
    uint64_t* totals;        // [G]; ~0 for a graph with invalid input
    uint64_t* ticks;         // [2G + 1]: [g] graph g finished, [G] batch start,
                             // [G + 1 + g] graph g started; or null
    BatchQueue* q;
    XcdWork* xw;             // [kMaxXcd]
    int32_t* big;            // [G] cooperative graphs in processing order (first q->nbig)
    int32_t* small;          // [G] workgroup graphs in processing order (first q->nsmall)
    int32_t* tiny;           // [G] wave graphs in processing order (first q->ntiny)
    char* xslots;            // kMaxXcd state slots (cooperative solves), xslot_bytes each
    char* wslots;            // one state slot per workgroup (graphs above lds_n)
    size_t slot_bytes;       // per-vertex state of one graph
    size_t xslot_bytes;      // slot_bytes + pair table
    int64_t nmax;            // vertices per graph the slots are sized for
    int64_t coop_edges;      // graphs with at least this many edges are cooperative (< 0: none)
    int lds_n;               // graphs with n <= lds_n keep their state in LDS
    int64_t wave_edges;      // graphs with m <= wave_edges and n <= wave_n: one wave each
    int wave_n;              //   (0: no wave graphs); wave_n = lds_n / waves per workgroup
    int hot_min;             // block tier of the segmented min: a label on at least this
                             //   many of a chunk's 64 sampled edge ends (0: off)
    int wave_min;            // wave tier: lanes sharing a label combine when at least
                             //   this many (0: off, every lane updates alone)
};

struct BatchLayout {
    size_t xw_off, lists_off, xslots_off, wslots_off, total;
};
BatchLayout batch_layout(int64_t G, int64_t nmax, int workgroups);

int launch_batch(const BatchArgs& A, int block, int workgroups, hipStream_t s);
size_t batch_slot_bytes(int64_t nmax);
size_t batch_xslot_bytes(int64_t nmax);
bool batch_allow_lds(int block, size_t bytes);
int batch_resident_workgroups(int block, size_t lds_bytes);

}  // namespace msf
