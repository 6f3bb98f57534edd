"""Statistics of a Filter-Borůvka pivot sample that feed the pivot network,
in float64 -- TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper's PivotSelection (Sec. V, Alg. 2) sorts a random sample of the
edges and takes an element of it; the library can instead let a small
network choose the sample quantile.  The network reads 16 numbers describing
the sample and the graph being split.  This module computes them from their
definitions, with L(w) = log2(1 + w) / 32:

  0-4   L of the sampled weight at sorted index floor(q * (s - 1)) for
        q = 0.10, 0.25, 0.50, 0.75, 0.90 (s = sample size).  The index is an
        integer decided in floating point: it is taken in single precision
        (q as a float, the product rounded to float, then truncated), the
        precision the device uses for it;
  5, 6  mean and (population) standard deviation of L over the sample;
  7     ties: the number of adjacent equal weights in the sorted sample,
        divided by s - 1 (0 for s = 1);
  8, 9  L of the smallest and of the largest sampled weight;
  10    log2(1 + c) / 32, c = current number of components;
  11    log2(1 + k) / 32, k = edges of the graph being split;
  12    log2(1 + k / max(c, 1)) / 8;
  13    recursion depth / 16;
  14    repeated endpoints: of the first min(s, 2048) draws, both endpoints of
        each drawn edge are listed; the number of adjacent equal entries of
        that list once sorted, divided by (list length - 1) (0 for a list of
        one entry);
  15    the constant 1.

No numbers here depend on the device: the oracle is float64 arithmetic on
the definitions above.
"""
from __future__ import annotations

import math

import numpy as np

QUANTILES = (0.10, 0.25, 0.50, 0.75, 0.90)
END_DRAWS = 2048


def level(w) -> float:
    """L(w) = log2(1 + w) / 32 for an integer weight."""
    return math.log2(1.0 + float(w)) / 32.0


def quantile_index(q: float, s: int) -> int:
    """floor(q * (s - 1)) taken in single precision (an integer decision the
    device makes in float)."""
    prod = np.float32(q) * np.float32(s - 1)
    return int(math.floor(float(prod)))


def adjacent_equal(sorted_values) -> int:
    """Number of i with sorted_values[i] == sorted_values[i + 1]."""
    a = list(sorted_values)
    return sum(1 for i in range(len(a) - 1) if a[i] == a[i + 1])


def pivot_features(weights, ends, comps: float, k: int, depth: int) -> np.ndarray:
    """The 16 features from the sampled weights (in draw order or sorted:
    they are sorted here), the endpoint list of the first draws (2 entries
    per draw, at most 2 * END_DRAWS), the current component count, the edge
    count of the graph being split and the recursion depth."""
    wsort = sorted(int(x) for x in weights)
    s = len(wsort)
    if s < 1:
        raise ValueError("empty sample")
    L = [level(x) for x in wsort]
    f = np.zeros(16, np.float64)
    for j, q in enumerate(QUANTILES):
        f[j] = L[quantile_index(q, s)]
    mean = sum(L) / s
    f[5] = mean
    f[6] = math.sqrt(sum((x - mean) ** 2 for x in L) / s)
    f[7] = adjacent_equal(wsort) / (s - 1) if s > 1 else 0.0
    f[8] = L[0]
    f[9] = L[-1]
    c = float(comps)
    f[10] = math.log2(1.0 + c) / 32.0
    f[11] = math.log2(1.0 + float(k)) / 32.0
    f[12] = math.log2(1.0 + float(k) / max(c, 1.0)) / 8.0
    f[13] = depth / 16.0
    e = sorted(int(x) for x in ends)
    f[14] = adjacent_equal(e) / (len(e) - 1) if len(e) > 1 else 0.0
    f[15] = 1.0
    return f


def sample_features(u, v, w, positions, comps: float, depth: int) -> np.ndarray:
    """Features of the sample drawn at `positions` (draw order) of the edge
    list (u, v, w) of the graph being split."""
    pos = np.asarray(positions, np.int64)
    ke = min(len(pos), END_DRAWS)
    ends = []
    for p in pos[:ke].tolist():
        ends.append(int(u[p]))
        ends.append(int(v[p]))
    return pivot_features(np.asarray(w)[pos], ends, comps, len(u), depth)
