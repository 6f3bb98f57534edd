"""Filter-Borůvka, step by step on the CPU (test infrastructure).

Follows the recursion of the paper's Alg. 2 (Sec. V):

    Rec-Filter-MST(E):
        if isSparse(E): base case (an MSF of E), record components
        pivot <- PivotSelection(E)
        E<= <- {e in E : key(e) <= pivot};  E> <- the rest
        Rec-Filter-MST(E<=)
        E>' <- heavy edges whose endpoints lie in different components
        Rec-Filter-MST(E>')

with the readings this library fixes where the paper leaves freedom:
  * keys are (w << 32 | edge id) and the split compares whole keys;
  * PivotSelection draws `sample` positions with replacement from the
    SplitMix64 stream mix(mix(seed) ^ (0x50495654 + split_index)), position
    floor(r * |E| / 2^64), sorts the sampled keys and takes the element at
    floor(q * (sample - 1));
  * isSparse: |E| < min_split, or 2|E| <= sparse_degree * (number of current
    components), or recursion depth >= 48;
  * a split with an empty side solves E directly.
The base case is Kruskal (the MSF of E is unique, so which algorithm finds
it does not matter); components are kept in a union-find, so representative
labels differ from the GPU's, which does not change any count or pivot.

Returns the MSF mask, total weight and one trace record per split, in the
depth-first order the recursion visits them; each record also holds the
pivot-network features of its sample (features.py), computed on the split's
edges named by their union-find representatives.
"""
from __future__ import annotations

import numpy as np

from . import kruskal
from .features import sample_features

GAMMA = 0x9E3779B97F4A7C15
MASK64 = (1 << 64) - 1
PIVOT_TAG = 0x50495654
MAX_DEPTH = 48


def _mix(z: int) -> int:
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def sample_positions(seed: int, split: int, length: int, sample: int) -> np.ndarray:
    base = _mix(_mix(seed) ^ (PIVOT_TAG + split))
    return np.array([(_mix((base + (i + 1) * GAMMA) & MASK64) * length) >> 64
                     for i in range(sample)], dtype=np.int64)


def pivot_index(q: float, sample: int) -> int:
    # q is single precision on the device; the index is taken in double
    idx = int(np.floor(float(np.float32(q)) * (sample - 1)))
    return min(max(idx, 0), sample - 1)


class _DSU:
    def __init__(self, n):
        self.p = list(range(n))

    def find(self, x):
        p = self.p
        while p[x] != x:
            p[x] = p[p[x]]
            x = p[x]
        return x

    def union(self, a, b):
        a, b = self.find(a), self.find(b)
        if a != b:
            self.p[a] = b


def filter_boruvka(u, v, w, n, seed=1, sample=4096, q=0.5, sparse_degree=4,
                   min_split=1 << 20, q_of_split=None):
    """q_of_split(i) may override the quantile per split (e.g. the values a
    learned pivot reported); default: q for every split."""
    u = np.asarray(u, np.int64)
    v = np.asarray(v, np.int64)
    w = np.asarray(w, np.uint64)
    m = len(u)
    ids = np.arange(m, dtype=np.int64)
    mask = np.zeros(m, np.uint8)
    dsu = _DSU(n)
    state = {"found": 0, "splits": 0}
    trace = []

    def base(a, b, ww, ii):
        bm, _, _ = kruskal(a.astype(np.int32), b.astype(np.int32), ww.astype(np.uint32), n)
        sel = np.nonzero(bm)[0]
        mask[ii[sel]] = 1
        for x, y in zip(a[sel].tolist(), b[sel].tolist()):
            dsu.union(x, y)
        state["found"] += len(sel)

    def rec(a, b, ww, ii, depth):
        k = len(a)
        if k == 0:
            return
        comps = n - state["found"]
        if k < min_split or 2 * k <= sparse_degree * comps or depth >= MAX_DEPTH:
            base(a, b, ww, ii)
            return
        split = state["splits"]
        state["splits"] += 1
        keys = (ww << np.uint64(32)) | ii.astype(np.uint64)
        pos = sample_positions(seed, split, k, sample)
        sk = np.sort(keys[pos])
        qq = q_of_split(split) if q_of_split else q
        pivot = int(sk[pivot_index(qq, sample)])
        light = keys <= np.uint64(pivot)
        nl = int(light.sum())
        rec_t = {"edges": k, "pivot": pivot, "light": nl, "kept": 0,
                 "features": sample_features(a, b, ww, pos, comps, depth)}
        trace.append(rec_t)
        if nl == 0 or nl == k:
            base(a, b, ww, ii)
            return
        hv = ~light
        ha, hb, hw, hi = a[hv], b[hv], ww[hv], ii[hv]
        rec(a[light], b[light], ww[light], ii[light], depth + 1)
        ra = np.array([dsu.find(x) for x in ha.tolist()], np.int64)
        rb = np.array([dsu.find(x) for x in hb.tolist()], np.int64)
        keep = ra != rb
        rec_t["kept"] = int(keep.sum())
        rec(ra[keep], rb[keep], hw[keep], hi[keep], depth + 1)

    rec(u, v, w, ids, 0)
    total = int(w[mask.astype(bool)].sum()) if m else 0
    return mask, total, trace
