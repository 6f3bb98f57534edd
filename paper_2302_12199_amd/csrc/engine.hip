// Borůvka round loop on one GPU (paper Sec. II-C; the while loop of Alg. 1).
//
// Each round: hook + 2-cycle break + MSF marking, pointer jumping, dense
// relabelling of the roots, then one streaming pass over the edges that
// relabels them, drops self-loops and runs the next round's lightest-edge
// search.  The host reads one small counter block per round (after the root
// scan, with the previous pass's live-edge count) to size the next launches;
// everything else stays on the device.
//
// Edge layout policy (all layouts keep position order = edge-id order):
//   * after round 0 the caller's arrays are rewritten once as label pairs
//     (16-bit packed when the next round has <= 65535 vertices), so later
//     passes gather from small label tables instead of the n-sized one;
//   * while most positions still hold live edges, later passes write nothing
//     and compose the label maps instead (parallel edges and self-loops are
//     cheap to skip, a rewrite is not);
//   * once fewer than half of the positions are live, the survivors are
//     compacted (stable, decoupled lookback).
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>

#include "engine.h"

namespace msf {

namespace {
constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }
constexpr double kCompactBelow = 0.5;   // compact when live / positions drops below this
constexpr int64_t kMax16 = 65535;       // label count that still fits the packed layout
constexpr int64_t kPreTailMinEdges = 1 << 23;   // smaller views are not worth renumbering
}  // namespace

size_t engine_carve(char* ws, int64_t m, int64_t n, EngineBuffers* B, bool buckets,
                    bool exact) {
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += align_up(bytes ? bytes : 1);
        return ws ? ws + o : nullptr;
    };
    const size_t nn = (size_t)(n > 0 ? n : 1), mm = (size_t)(m > 0 ? m : 1);
    const int64_t tile_min = kTile < kRelabelTile ? kTile : kRelabelTile;
    const size_t tiles = (size_t)((std::max<int64_t>(m, n) + tile_min - 1) / tile_min) + 1;
    EngineBuffers b;
    b.ctrl = (Ctrl*)take(sizeof(Ctrl));
    b.status = (uint64_t*)take(tiles * 8);
    b.cflags = (uint64_t*)take(((mm + kRelabelTile - 1) / kRelabelTile) * (kRelabelTile / 8));
    b.cbsum = (uint64_t*)take(1024 * 8);
    for (int i = 0; i < 2; ++i) b.best[i] = (uint64_t*)take(nn * 8);
    b.parent = (int32_t*)take(nn * 4);
    b.rootbits = (uint64_t*)take((nn / 64 + 1) * 8);
    b.livebits = (uint64_t*)take((nn / 64 + 1) * 8);
    for (int i = 0; i < 2; ++i) b.lab[i] = (int32_t*)take(nn * 4);
    for (int i = 0; i < 2; ++i) b.map[i] = (int32_t*)take(nn * 4);
    for (int i = 0; i < 2; ++i) b.orig[i] = (int32_t*)take(nn * 4);
    b.f32u = (int32_t*)take(mm * 4);
    b.f32v = (int32_t*)take(mm * 4);
    b.p16 = (uint32_t*)take(mm * 4);
    for (int i = 0; i < 2; ++i) {
        b.cbuf[i].u = (int32_t*)take(mm * 4);
        b.cbuf[i].v = (int32_t*)take(mm * 4);
        b.cbuf[i].w = (uint32_t*)take(mm * 4);
        b.cbuf[i].id = (uint32_t*)take(mm * 4);
    }
    const size_t slots = (size_t)kTailMax * (kTailMax - 1) / 2;
    b.pairs = (uint64_t*)take(slots * 8);
    b.perm = (int32_t*)take((size_t)kTailMax * 4);
    for (int i = 0; i < 2; ++i) {
        b.list_xy[i] = (uint32_t*)take(slots * 4);
        b.list_key[i] = (uint64_t*)take(slots * 8);
    }
    b.dpair = b.dmin = nullptr;
    b.dslots = 0;
    if (exact) {   // a power of two of at least twice the edges: probing always ends
        int64_t sl = 1024;
        while (sl < 2 * (int64_t)mm) sl <<= 1;
        b.dslots = sl;
        b.dpair = (uint64_t*)take((size_t)sl * 8);
        b.dmin = (uint64_t*)take((size_t)sl * 8);
    }
    if (buckets) off += bucket_carve(ws ? ws + off : nullptr, m, n, &b.bk);
    else b.bk = BucketBuffers{};
    b.round0 = MSF_ROUND0_AUTO;
    b.dedup = MSF_DEDUP_AUTO;
    b.tail = 0;
    b.ncap = n;
    b.mcap = m;
    if (B) *B = b;
    return off;
}

size_t engine_bytes(int64_t m, int64_t n, bool buckets, bool exact) {
    return engine_carve(nullptr, m, n, nullptr, buckets, exact);
}

static bool aligned16(const View& g) {
    return ((((uintptr_t)g.u | (uintptr_t)g.v | (uintptr_t)g.w | (uintptr_t)g.p16 |
              (uintptr_t)g.id) & 15) == 0);
}

static double view_read_bytes(int mode) { return mode == kFull16 ? 8.0 : 12.0; }

int engine_solve(EngineBuffers& B, int mode, const View& view0, int64_t nv, uint8_t* mask,
                 int32_t* rep, hipStream_t s, msf_stats* stats, int32_t hot) {
    Ctrl* hc = host_ctrl();
    Ctrl* dc = B.ctrl;
    View view = view0;
    const int32_t* cmap = nullptr;   // stored labels -> this round's labels (null: identity)
    int64_t nc = nv;                 // size of the stored-label space
    int cur = 0, labsel = 0, mapsel = 0, cbsel = 0, origsel = 0;
    int64_t nr = nv;
    int st;

    // Round 0 lightest edges (on the caller's arrays, or on a compact view
    // whose positions are already in id order).
    // Large graphs on the caller's arrays without id locality: round 0 by
    // vertex buckets (with locality the edge-list round 0 mostly hits in L2).
    // Both choices below read one sample of 4096 evenly spaced edges: do at
    // least half of them join ids less than 2^14 apart (locality)?
    const bool can_bucket = mode == kOrig && aligned16(view) &&
                            bucket_usable(B.bk, view.len, nv);
    bool local = false;
    if (mode == kOrig && view.len >= kLocalitySample &&
        ((can_bucket && B.round0 == MSF_ROUND0_AUTO) || B.dedup == MSF_DEDUP_AUTO)) {
        bucket_sample_locality(view.u, view.v, view.len, dc, s);
        HIP_TRY(hipGetLastError());
        if ((st = read_ctrl(dc, hc, s))) return st;
        local = hc->aux[0] * 2 >= (uint64_t)kLocalitySample;
    }
    bool bucketed = can_bucket && (B.round0 != MSF_ROUND0_AUTO || !local);
    // Parallel-edge removal at every compaction, and compaction from round 0
    // on (where round 0 runs on the edge list): contracted components of a
    // graph with locality share many edges, so each round shrinks the next.
    const int dedup = B.dedup == MSF_DEDUP_EXACT && B.dslots > 0 ? kDedupExact
                      : B.dedup == MSF_DEDUP_LOCAL || B.dedup == MSF_DEDUP_EXACT ||
                              (B.dedup == MSF_DEDUP_AUTO && local)
                          ? kDedupLocal
                          : kDedupNone;
    // Every round's minima also say which end of its edge the vertex is (up
    // to 2^31 positions: the position takes 31 bits, the side one), so the
    // hook reads only the other end.  The bucketed path takes m < 2^31.
    const bool side_keys = view.len <= kSideKeyMaxEdges;
    int h = -1;
    if (bucketed) {
        bucket_minedge(B.bk, view.u, view.v, view.w, view.len, nv, B.best[cur], dc, s);
    } else {
        h = prof_begin(K_FILL, s);
        launch_fill_u64(B.best[cur], nr, kKeyMax, s);
        prof_end(h, s, 8.0 * nr);
        h = prof_begin(K_MINEDGE_R0, s);
        launch_minedge_r0(view.u, view.v, view.w, view.len, nv, B.best[cur], dc, hot, local,
                          side_keys, s);
        prof_end(h, s, 12.0 * view.len + 8.0 * nv);
    }
    HIP_TRY(hipGetLastError());
    // Edges with ids out of range were skipped by the lightest-edge search (no
    // minimum holds them), so the first round runs on valid edges only; the
    // error bit is read with that round's counters.

    // The live-edge count of a relabelling pass is read with the next round's
    // counters (one host synchronisation per round): a pass that leaves no
    // live edge leaves every minimum empty, so that round finds nothing.
    int64_t m_live = view.len;
    bool m_pending = false, m_compacted = false;
    uint32_t rounds = stats ? stats->rounds : 0;
    const uint32_t first_round = rounds;
    while (m_live > 0 || m_pending) {
        launch_scan_prep(B.status, 0, dc, 1, s);
        const int hh = prof_begin(K_HOOK, s);
        launch_hook(mode, B.best[cur], nr, view, cmap, B.parent, mask, B.rootbits, B.livebits,
                    dc, side_keys, s);
        prof_end(hh, s, 12.25 * nr);   // best[] in; parent[], root and live bits out
        int32_t* lab = B.lab[labsel];
        for (int attempt = 0;; ++attempt) {
            h = prof_begin(K_JUMP, s);
            launch_jump(B.parent, nr, 16, dc, s);
            prof_end(h, s, 12.0 * nr);
            const int64_t ntv = (nr + kTile - 1) / kTile;
            launch_scan_prep(B.status, ntv, dc, 0, s);
            h = prof_begin(K_SCAN_ROOTS, s);
            launch_scan_roots(B.rootbits, nr, lab, B.status, dc, s);
            prof_end(h, s, 0.125 * nr);   // root bits in (+ a label per root)
            h = prof_begin(K_LABEL, s);
            launch_label(B.parent, B.livebits, nr, lab, B.best[cur ^ 1], dc, s);
            prof_end(h, s, 8.125 * nr);   // parent[] and live bits in, label[] out (+ best_next)
            HIP_TRY(hipGetLastError());
            if ((st = read_ctrl(dc, hc, s))) return st;
            if (!hc->jump_more) break;
            if (attempt > 64) {
                set_err_text("pointer jumping did not converge");
                return MSF_EINTERNAL;
            }
            launch_zero_bytes((uint8_t*)&dc->jump_more, sizeof(uint32_t), s);
        }
        if (hc->err & kErrRange) return MSF_ERANGE;
        if (hc->err) {
            char buf[96];
            snprintf(buf, sizeof buf, "device error bits 0x%x in round %u", hc->err, rounds);
            set_err_text(buf);
            return MSF_EINTERNAL;
        }
        if (m_pending) {
            m_pending = false;
            m_live = (int64_t)hc->m_next;
            if (m_compacted) {     // only a compaction changes the number of positions
                view.len = m_live;
                prof_add(K_COMPACT, 16.0 * m_live);
            }
            if (m_live == 0) break;
        }
        const uint64_t live = hc->live, found = hc->found;
        const int64_t nn = (int64_t)hc->n_next;
        // Before the bucketed relabelling pass: the round-1 labels on many
        // edge ends are renumbered first (their minima then stay in LDS).
        // The single-workgroup tail takes over the next rounds once few labels
        // are left and its pair list is short: automatically at <= kTailMax
        // labels with at most kTailAutoPairs possible pairs (live edges or
        // label pairs, whichever is fewer), else at the caller's threshold.
        const int64_t max_pairs =
            nn <= kTailMax ? std::min<int64_t>(m_live, nn * (nn - 1) / 2) : INT64_MAX;
        const bool tail_next = B.tail > 0 ? nn <= B.tail
                                          : nn <= kTailMax && max_pairs <= kTailAutoPairs;
        if (bucketed && mode == kOrig && !tail_next)
            bucket_hot_first(B.bk, view.u, view.v, view.len, lab, nr, nn, s);
        // Before the tail: the labels of its vertices are renumbered hot first
        // (the pair pass keeps the pairs among the first ones in LDS).
        const bool pre_tail_hot = tail_next && view.len >= kPreTailMinEdges;
        if (pre_tail_hot && nn > kPairHot)
            launch_hot_first_small(mode, view, cmap, lab, nr, nn, B.perm, &dc->aux[2], s);
        else if (pre_tail_hot)   // every pair fits the LDS table
            launch_fill_u64(&dc->aux[2], 1, (uint64_t)nn, s);
        prof_add(K_HOOK, (side_keys ? 13.0 : 17.0) * live);   // other end(s), best[other], mask
        prof_add(K_SCAN_ROOTS, 4.0 * nn);
        prof_add(K_LABEL, 8.0 * nn);
        if (stats && rounds < MSF_MAX_TRACE) {
            stats->round_live[rounds] = live;
            stats->round_edges[rounds] = (uint64_t)m_live;
            stats->round_found[rounds] = found;
            stats->round_vertices[rounds] = (uint64_t)nr;
        }
        ++rounds;

        if (rep) {
            launch_rep_update(B.parent, B.livebits, lab, nr, rounds - 1 == first_round ? nullptr : B.orig[origsel],
                              B.orig[origsel ^ 1], rep, s);
            origsel ^= 1;
        }

        // M: stored labels -> next-round labels.
        const int32_t* M = lab;
        if (cmap) {
            h = prof_begin(K_COMPOSE, s);
            launch_compose(cmap, nc, lab, B.map[mapsel], s);
            prof_end(h, s, 12.0 * nc);
            M = B.map[mapsel];
            mapsel ^= 1;
        }
        // the streaming pass uses 16-byte vector loads
        const bool aligned = ((((uintptr_t)view.u | (uintptr_t)view.v | (uintptr_t)view.w |
                                (uintptr_t)view.p16 | (uintptr_t)view.id) & 15) == 0);
        if (nn <= 1) break;        // one component left: every remaining edge is a self-loop
        if (tail_next && aligned) {
            // Last pass keeps the lightest edge per vertex pair; one workgroup
            // then finishes all remaining rounds.
            const int64_t slots = nn * (nn - 1) / 2;
            h = prof_begin(K_PASS, s);
            launch_fill_u64(B.pairs, slots, kKeyMax, s);
            if (!launch_pass(mode, kOutNone, view, M, nc, B.f32u, B.f32v, B.p16, B.best[cur ^ 1],
                             nn, B.pairs, pre_tail_hot ? &dc->aux[2] : nullptr, dc, side_keys,
                             s)) {
                set_err_text("unsupported pass layout");
                return MSF_EINTERNAL;
            }
            prof_end(h, s, view_read_bytes(mode) * view.len + 8.0 * m_live + 8.0 * slots);
            h = prof_begin(K_TAIL, s);
            launch_tail(B.pairs, nn, B.list_xy, B.list_key, mode == kCompact ? view.id : nullptr,
                        mask, rep ? B.orig[origsel] : nullptr, rep, dc, s);
            prof_end(h, s, 16.0 * slots);
            HIP_TRY(hipGetLastError());
            if ((st = read_ctrl(dc, hc, s))) return st;
            if (hc->err) {
                set_err_text("device error bits in the tail");
                return MSF_EINTERNAL;
            }
            for (uint32_t t = 0; t < hc->tail_rounds; ++t) {
                if (stats && rounds < MSF_MAX_TRACE) {
                    stats->round_live[rounds] = hc->tail_live[t];
                    stats->round_edges[rounds] = hc->tail_scan[t];
                    stats->round_found[rounds] = hc->tail_found[t];
                    stats->round_vertices[rounds] = t == 0 ? (uint64_t)nn : hc->tail_live[t];
                }
                ++rounds;
            }
            break;
        }
        const bool compact = !aligned || (dedup != kDedupNone && !bucketed) ||
                             (dedup != kDedupNone && mode != kOrig) ||
                             (mode != kOrig && (double)m_live < kCompactBelow * (double)view.len);
        View next = view;
        int next_mode = mode;
        const int32_t* next_cmap = nullptr;
        int64_t next_nc = nn;
        launch_fill_u64(&dc->m_next, 1, 0, s);
        if (compact) {
            EdgeSoA out = B.cbuf[cbsel];
            cbsel ^= 1;
            if (dedup == kDedupExact) {   // the lightest key of every vertex pair
                h = prof_begin(K_DEDUP, s);
                launch_fill_u64(B.dpair, B.dslots, kKeyMax, s);
                launch_fill_u64(B.dmin, B.dslots, kKeyMax, s);
                launch_dedup_insert(mode, view, M, B.dpair, B.dmin, B.dslots, s);
                prof_end(h, s, 16.0 * B.dslots + view_read_bytes(mode) * view.len + 8.0 * m_live);
            }
            h = prof_begin(K_COMPACT, s);
            launch_compact(mode, view, M, out, B.best[cur ^ 1], nn, B.cflags, B.status, B.cbsum,
                           dc, dedup, B.dpair, B.dmin, B.dslots, local, side_keys, s);
            prof_end(h, s, view_read_bytes(mode) * view.len + 8.0 * m_live);
            next.u = out.u; next.v = out.v; next.w = out.w; next.id = out.id; next.p16 = nullptr;
            next_mode = kCompact;
        } else {
            int out = kOutNone;
            if (mode == kOrig) out = nn <= kMax16 ? kOut16 : kOut32;
            else if (mode == kFull32 && nn <= kMax16) out = kOut16;
            if (bucketed && mode == kOrig) {
                bucket_relabel(B.bk, view.w, view.len, nv, M, out, B.f32u,
                               B.f32v, B.p16, B.best[cur ^ 1], nn, dc, s);
            } else {
                h = prof_begin(mode == kOrig ? K_PASS_R0 : K_PASS, s);
                if (!launch_pass(mode, out, view, M, nc, B.f32u, B.f32v, B.p16, B.best[cur ^ 1],
                                 nn, nullptr, nullptr, dc, side_keys, s)) {
                    set_err_text("unsupported pass layout");
                    return MSF_EINTERNAL;
                }
                prof_end(h, s, view_read_bytes(mode) * view.len + 8.0 * m_live +
                                   (out == kOut32 ? 8.0 : out == kOut16 ? 4.0 : 0.0) * view.len +
                                   8.0 * nn);
            }
            if (out == kOut32) {
                next.u = B.f32u; next.v = B.f32v; next.p16 = nullptr; next_mode = kFull32;
            } else if (out == kOut16) {
                next.p16 = B.p16; next.u = next.v = nullptr; next_mode = kFull16;
            } else {
                next_cmap = M;
                next_nc = nc;
            }
        }
        HIP_TRY(hipGetLastError());
        m_pending = true;
        m_compacted = compact;
        view = next;
        mode = next_mode;
        cmap = next_cmap;
        nc = next_nc;
        nr = nn;
        cur ^= 1;
        labsel ^= 1;
        if (rounds - first_round > 70) {
            set_err_text("too many rounds");
            return MSF_EINTERNAL;
        }
    }
    if (stats) stats->rounds = rounds;
    return MSF_OK;
}

}  // namespace msf
