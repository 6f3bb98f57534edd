// Host-side launchers of the device kernels (each in the .hip file that
// defines the kernel).  All take the stream to launch on.
#pragma once
#include "common.h"

namespace msf {

// boruvka.hip
void launch_fill_u64(uint64_t* p, int64_t n, uint64_t val, hipStream_t s);
void launch_zero_bytes(uint8_t* p, int64_t n, hipStream_t s);
void launch_scan_prep(uint64_t* status, int64_t ntiles, Ctrl* ctrl, int round_begin,
                      hipStream_t s);
// local: the edges join nearby ids (locality sample); then the minima of a
// sliding window of ids are taken in LDS.
// side_keys (taken when m <= kSideKeyMaxEdges): best[] gets w << 32 |
// position << 1 | side (side 1: the vertex is the edge's v end), which the
// hook reads to fetch only the other end; else w << 32 | position.
constexpr int64_t kSideKeyMaxEdges = 1ll << 31;
void launch_minedge_r0(const int32_t* u, const int32_t* v, const uint32_t* w, int64_t m,
                       int64_t n, uint64_t* best, Ctrl* ctrl, int32_t hot, bool local,
                       bool side_keys, hipStream_t s);
// side_keys: best[] holds w << 32 | position << 1 | side, else w << 32 |
// position (the form every kernel that fills best[] was given).
// rootbits / livebits ((nr + 63) / 64 words each): bit x says whether x is a
// root that found an edge / found an edge at all.
void launch_hook(int mode, const uint64_t* best, int64_t nr, const View& g, const int32_t* cmap,
                 int32_t* parent, uint8_t* mask, uint64_t* rootbits, uint64_t* livebits,
                 Ctrl* ctrl, bool side_keys, hipStream_t s);
void launch_jump(int32_t* parent, int64_t nr, int iters, Ctrl* ctrl, hipStream_t s);
void launch_scan_roots(const uint64_t* rootbits, int64_t nr, int32_t* label,
                       uint64_t* status, Ctrl* ctrl, hipStream_t s);
void launch_label(const int32_t* parent, const uint64_t* livebits, int64_t nr, int32_t* label,
                  uint64_t* best_next, const Ctrl* ctrl, hipStream_t s);
void launch_compose(const int32_t* cmap, int64_t nc, const int32_t* label, int32_t* out,
                    hipStream_t s);
// side_keys: the next round's minima as side keys (see launch_minedge_r0);
// the pair table before the tail always holds w << 32 | position.
bool launch_pass(int in_mode, int out, const View& g, const int32_t* M, int64_t nc, int32_t* ou,
                 int32_t* ov, uint32_t* op16, uint64_t* best_next, int64_t nn, uint64_t* pairs,
                 const uint64_t* pair_hot, Ctrl* ctrl, bool side_keys, hipStream_t s);
// Before the tail: this round's labels lab[0, nr) (values in [0, nn), nn <= the
// tail's limit) renumbered hot first; *hot = the number of hot labels.
void launch_hot_first_small(int mode, const View& g, const int32_t* cmap, int32_t* lab, int64_t nr,
                            int64_t nn, int32_t* perm, uint64_t* hot, hipStream_t s);
// tail.hip
void launch_tail(const uint64_t* pairs, int64_t nn, uint32_t* const list_xy[2],
                 uint64_t* const list_key[2], const uint32_t* view_id, uint8_t* mask,
                 const int32_t* orig_in, int32_t* rep, Ctrl* ctrl, hipStream_t s);
void launch_rep_update(const int32_t* parent, const uint64_t* livebits, const int32_t* label,
                       int64_t nr, const int32_t* orig_cur, int32_t* orig_next, int32_t* rep,
                       hipStream_t s);
// dedup (DedupKind): kDedupLocal keeps only the lightest edge per vertex pair
// within each tile; kDedupExact keeps the edge whose key the global table
// (dpair, dmin; dslots entries, filled by launch_dedup_insert) holds for its pair.
// flags: one bit per position (tiles of 2048 positions); cnt: a word per tile;
// bsum: kScanTop words.  ctrl->m_next receives the number of kept edges.
// best_next holds nn entries (side keys when side_keys); local: the graph has
// id locality (the next round's minima are then taken in a sliding LDS window
// of labels).
void launch_compact(int in_mode, const View& g, const int32_t* M, EdgeSoA out,
                    uint64_t* best_next, int64_t nn, uint64_t* flags, uint64_t* cnt,
                    uint64_t* bsum, Ctrl* ctrl, int dedup, const uint64_t* dpair,
                    const uint64_t* dmin, int64_t dslots, bool local, bool side_keys,
                    hipStream_t s);
// filter.hip: exclusive scan of per-tile counts in place (nt <= 2^21 tiles;
// bsum holds kScanTop chunk sums), the total to *total.
void launch_scan_tiles(uint64_t* cnt, uint32_t nt, uint64_t* bsum, uint64_t* total,
                       hipStream_t s);
// Global pair table of exact parallel-edge removal: every live relabelled edge
// enters its vertex pair and min-reduces its key.  dpair/dmin must hold kKeyMax.
void launch_dedup_insert(int in_mode, const View& g, const int32_t* M, uint64_t* dpair,
                         uint64_t* dmin, int64_t dslots, hipStream_t s);

}  // namespace msf
