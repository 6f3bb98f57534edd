"""Filter-Borůvka's per-split trace from set definitions -- TEST
INFRASTRUCTURE ONLY (see the package docstring).

A second, independent formulation of the split trace that filter_ref.py
records while it runs the recursion of the paper's Alg. 2 (Sec. V) with a
union-find.  Here nothing is carried from split to split; every quantity is
recomputed from the input graph with a library connected-components routine.
It rests on one fact about the recursion: edges are finished in key order.
Each recursive call owns a key interval (lo, hi]; when it starts, every edge
with key <= lo has been handled, so the current components are exactly the
connected components of G_lo = (V, {e : key(e) <= lo}) and the number of
components is that count (isolated vertices included).  Then, for the call
owning (lo, hi]:

  * its edges are those with key in (lo, hi] whose endpoints lie in different
    components of G_lo (at the top, lo = -inf, every edge, self-loops too),
    in edge-id order, each endpoint named by its component;
  * the pivot is the sample quantile of those edges' keys (the readings of
    PivotSelection fixed in filter_ref.py);
  * light = edges with key <= pivot; the light call owns (lo, pivot];
  * kept = heavy edges (key in (pivot, hi]) whose endpoints lie in different
    components of G_pivot (the Filter step, Sec. V: an edge inside a
    component of the lighter edges cannot be in the MSF, by the cycle
    property); the heavy call owns (pivot, hi] and its edges are exactly
    these.

The isSparse rule, the degenerate-split rule and the depth cap are those of
filter_ref.py.
"""
from __future__ import annotations

import numpy as np
from scipy.sparse import coo_matrix
from scipy.sparse.csgraph import connected_components

from .features import sample_features
from .filter_ref import MAX_DEPTH, pivot_index, sample_positions


def components_below(u, v, keys, n, bound):
    """(labels, count) of the connected components of (V, {e : key <= bound})."""
    sel = keys <= np.uint64(bound)
    a, b = u[sel], v[sel]
    g = coo_matrix((np.ones(len(a)), (a, b)), shape=(n, n))
    count, labels = connected_components(g, directed=False)
    return labels.astype(np.int64), int(count)


def trace_by_definition(u, v, w, n, seed=1, sample=4096, q=0.5, sparse_degree=4,
                        min_split=1 << 20, q_of_split=None):
    """List of split records {edges, pivot, light, kept, features} in the
    depth-first order of the recursion."""
    u = np.asarray(u, np.int64)
    v = np.asarray(v, np.int64)
    w = np.asarray(w, np.uint64)
    m = len(u)
    keys = (w << np.uint64(32)) | np.arange(m, dtype=np.uint64)
    trace = []

    def call(lo, hi, depth):
        in_range = np.ones(m, bool) if hi is None else keys <= np.uint64(hi)
        if lo is None:
            comp, comps = np.arange(n, dtype=np.int64), n
        else:
            in_range &= keys > np.uint64(lo)
            comp, comps = components_below(u, v, keys, n, lo)
            in_range &= comp[u] != comp[v]
        idx = np.nonzero(in_range)[0]
        k = len(idx)
        if k == 0:
            return
        if k < min_split or 2 * k <= sparse_degree * comps or depth >= MAX_DEPTH:
            return
        split = len(trace)
        pos = sample_positions(seed, split, k, sample)
        qq = q_of_split(split) if q_of_split else q
        pivot = int(np.sort(keys[idx[pos]])[pivot_index(qq, sample)])
        light = int((keys[idx] <= np.uint64(pivot)).sum())
        rec = {"edges": k, "pivot": pivot, "light": light, "kept": 0,
               "features": sample_features(comp[u[idx]], comp[v[idx]], w[idx], pos, comps,
                                           depth)}
        trace.append(rec)
        if light == 0 or light == k:
            return
        call(lo, pivot, depth + 1)
        comp_p, _ = components_below(u, v, keys, n, pivot)
        heavy = idx[keys[idx] > np.uint64(pivot)]
        rec["kept"] = int((comp_p[u[heavy]] != comp_p[v[heavy]]).sum())
        call(pivot, hi, depth + 1)

    call(None, None, 0)
    return trace
