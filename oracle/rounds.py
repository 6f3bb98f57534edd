"""Plain Borůvka rounds, one at a time (test infrastructure).

Restates the sequential round of the paper (Sec. II-C): every vertex picks its
lightest incident edge; the picked edges join vertices into components, all
picked edges are MSF edges (cut property); each component becomes one vertex;
edges are relabelled and self-loops dropped.  Parallel edges are kept (the
paper makes their removal optional), so the per-round edge counts here are
the ones a solver without parallel-edge removal sees.

Components are found with a library connected-components routine on the
picked edges, i.e. by definition, not by pointer jumping.
"""
from __future__ import annotations

import numpy as np
from scipy.sparse import coo_matrix
from scipy.sparse.csgraph import connected_components

MAXKEY = np.uint64(2**64 - 1)


def boruvka_rounds(u, v, w, n):
    """Returns (mask, total, rounds) where rounds is a list of dicts with
    ``live`` (vertices with an incident non-self-loop edge), ``edges``
    (non-self-loop edges entering the round), ``pairs`` (distinct vertex
    pairs among them: the edges left once parallel edges are removed),
    ``vertices`` (vertex labels of the round) and ``found`` (MSF edges picked
    in the round)."""
    u = np.asarray(u, np.int64)
    v = np.asarray(v, np.int64)
    w = np.asarray(w, np.uint64)
    m = len(u)
    eid = np.arange(m, dtype=np.uint64)
    key = (w << np.uint64(32)) | eid
    keep = u != v
    cu, cv, ck = u[keep], v[keep], key[keep]
    nr = n
    mask = np.zeros(m, np.uint8)
    rounds = []
    while len(cu) > 0:
        best = np.full(nr, MAXKEY, dtype=np.uint64)
        np.minimum.at(best, cu, ck)
        np.minimum.at(best, cv, ck)
        live = best != MAXKEY
        picked = np.unique(best[live])          # each picked edge once
        pe = (picked & np.uint64(0xFFFFFFFF)).astype(np.int64)
        mask[pe] = 1
        # endpoints of the picked edges in the current labelling
        pos = np.searchsorted(ck, picked, sorter=np.argsort(ck))
        order = np.argsort(ck)
        pidx = order[pos]
        a, b = cu[pidx], cv[pidx]
        g = coo_matrix((np.ones(len(a)), (a, b)), shape=(nr, nr))
        ncomp, comp = connected_components(g, directed=False)
        # only components that contain a live vertex survive as vertices
        live_comp = np.zeros(ncomp, bool)
        live_comp[comp[live]] = True
        newid = np.cumsum(live_comp) - 1
        lo, hi = np.minimum(cu, cv), np.maximum(cu, cv)
        rounds.append({"live": int(live.sum()), "edges": int(len(cu)),
                       "pairs": int(len(np.unique(lo * nr + hi))), "vertices": int(nr),
                       "found": int(len(picked))})
        lu, lv = newid[comp[cu]], newid[comp[cv]]
        k2 = lu != lv
        cu, cv, ck = lu[k2], lv[k2], ck[k2]
        nr = int(live_comp.sum())
    total = int(w[mask.astype(bool)].sum()) if m else 0
    return mask, total, rounds
