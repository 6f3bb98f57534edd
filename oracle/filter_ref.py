"""Filter-Borůvka, step by step on the CPU (test infrastructure).

Follows the recursion of the paper's Alg. 2 (Sec. V):

    Rec-Filter-MST(E):
        if isSparse(E): base case (an MSF of E), record components
        pivot <- PivotSelection(E)
        E<= <- {e in E : key(e) <= pivot};  E> <- the rest
        Rec-Filter-MST(E<=)
        E>' <- heavy edges whose endpoints lie in different components
        Rec-Filter-MST(E>')

Two variants the paper names, both off by default:
  * balanced-split retry (proof of Thm. 1: repeat the pivot selection until
    the split is balanced): with `retries` > 0 a split is accepted when its
    light fraction lies within 1/6 of the target quantile (for the median:
    both sides in [|E|/3, 2|E|/3], the paper's band); otherwise the sample is
    drawn again from the next stream of the same split, at most `retries`
    more times, and the last draw is used if none was balanced;
  * deferral of small filtered sets (Sec. VI-C, further remarks): a call at
    depth >= 1 whose filtered heavy set has fewer than `defer` edges does not
    recurse on it but returns it to the calling level, which filters it again
    together with, and before, that level's own heavy edges; edges a right
    recursion hands back are treated like that call's own filtered set.

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


def stream_base(seed: int, split: int, attempt: int = 0) -> int:
    """Stream of draw `attempt` of split `split`: the first draw uses
    mix(mix(seed) ^ (tag + split)); a redraw a >= 1 uses mix(that + a * GAMMA)."""
    base = _mix(_mix(seed) ^ (PIVOT_TAG + split))
    return base if attempt == 0 else _mix((base + attempt * GAMMA) & MASK64)


def sample_positions(seed: int, split: int, length: int, sample: int,
                     attempt: int = 0) -> np.ndarray:
    base = stream_base(seed, split, attempt)
    return np.array([(_mix((base + (i + 1) * GAMMA) & MASK64) * length) >> 64
                     for i in range(sample)], dtype=np.int64)


def balanced(light: int, total: int, q: float) -> bool:
    """The retry's acceptance band: light / total within 1/6 of q, tested as
    (6q - 1) total <= 6 light <= (6q + 1) total (q in single precision, the
    test in double, as the library's host code decides it; exact for the
    median)."""
    qq = float(np.float32(q))
    return (6.0 * qq - 1.0) * total <= 6.0 * light <= (6.0 * qq + 1.0) * total


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
                   min_split=1 << 20, q_of_split=None, retries=0, defer=0, info=None):
    """q_of_split(i) may override the quantile per split (e.g. the values a
    learned pivot reported); default: q for every split.  retries and defer
    switch on the two variants above.  `info`, a dict, receives the counts
    of base cases, redraws and deferrals."""
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
        state["base_cases"] += 1
        bm, _, _ = kruskal(a.astype(np.int32), b.astype(np.int32), ww.astype(np.uint32), n)
        sel = np.nonzero(bm)[0]
        mask[ii[sel]] = 1
        for x, y in zip(a[sel].tolist(), b[sel].tolist()):
            dsu.union(x, y)
        state["found"] += len(sel)

    empty = (np.zeros(0, np.int64), np.zeros(0, np.int64), np.zeros(0, np.uint64),
             np.zeros(0, np.int64))

    def filt(a, b, ww, ii):
        """Heavy edges named by their representatives; those inside one
        component are dropped (the Filter step)."""
        ra = np.array([dsu.find(x) for x in a.tolist()], np.int64)
        rb = np.array([dsu.find(x) for x in b.tolist()], np.int64)
        keep = ra != rb
        return ra[keep], rb[keep], ww[keep], ii[keep]

    def rec(a, b, ww, ii, depth):
        """Solves the call's edges; returns the edges it defers to its caller."""
        k = len(a)
        if k == 0:
            return empty
        comps = n - state["found"]
        if k < min_split or 2 * k <= sparse_degree * comps or depth >= MAX_DEPTH:
            base(a, b, ww, ii)
            return empty
        split = state["splits"]
        state["splits"] += 1
        keys = (ww << np.uint64(32)) | ii.astype(np.uint64)
        qq = q_of_split(split) if q_of_split else q
        for attempt in range(retries + 1):
            pos = sample_positions(seed, split, k, sample, attempt)
            sk = np.sort(keys[pos])
            pivot = int(sk[pivot_index(qq, sample)])
            light = keys <= np.uint64(pivot)
            nl = int(light.sum())
            if retries == 0 or attempt == retries or balanced(nl, k, qq):
                break
            state["retries"] += 1
        rec_t = {"edges": k, "pivot": pivot, "light": nl, "kept": 0, "attempts": attempt + 1,
                 "deferred_in": 0, "features": sample_features(a, b, ww, pos, comps, depth)}
        trace.append(rec_t)
        if nl == 0 or nl == k:
            base(a, b, ww, ii)
            return empty
        hv = ~light
        ha, hb, hw, hi = a[hv], b[hv], ww[hv], ii[hv]
        da, db, dw, di = rec(a[light], b[light], ww[light], ii[light], depth + 1)
        rec_t["deferred_in"] = len(da)
        # the deferred edges first: their keys lie below the heavy ones
        parts = [filt(da, db, dw, di), filt(ha, hb, hw, hi)]
        ka, kb, kw, ki = (np.concatenate([p[j] for p in parts]) for j in range(4))
        rec_t["kept"] = len(ka)
        while len(ka):
            if depth > 0 and len(ka) < defer:
                state["deferrals"] += 1
                return ka, kb, kw, ki
            ka, kb, kw, ki = rec(ka, kb, kw, ki, depth + 1)
        return empty

    state.update(deferrals=0, retries=0, base_cases=0)
    rec(u, v, w, ids, 0)
    if info is not None:
        info.update(base_cases=state["base_cases"], retries=state["retries"],
                    deferrals=state["deferrals"])
    total = int(w[mask.astype(bool)].sum()) if m else 0
    return mask, total, trace
