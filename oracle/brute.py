"""Brute-force and by-definition MSF oracles for tiny inputs (test infrastructure).

Both follow the problem statement of the paper (Sec. II-B: an MST of every
connected component) with ties broken by edge id (Sec. II-C).
"""
from __future__ import annotations

import itertools

import numpy as np


def _find(p, x):
    while p[x] != x:
        x = p[x]
    return x


def brute_force(u, v, w, n):
    """Enumerate every spanning forest; return the mask of the minimum one.

    The MSF has n - c edges (c = number of components).  Among all acyclic
    edge subsets of that size, the one minimising sum(w_e * 2^32 + e) is the
    minimum-weight forest with ties broken by edge id: the perturbed weights
    are distinct and order edges exactly as (w, id) does.  Exponential; meant
    for n <= 8 and m <= ~16.
    """
    m = len(u)
    p = list(range(n))
    for a, b in zip(u, v):
        ra, rb = _find(p, int(a)), _find(p, int(b))
        if ra != rb:
            p[ra] = rb
    c = sum(1 for x in range(n) if _find(p, x) == x)
    k = n - c
    cand = [e for e in range(m) if u[e] != v[e]]
    best, best_set = None, ()
    for sub in itertools.combinations(cand, k):
        q = list(range(n))
        ok = True
        for e in sub:
            ra, rb = _find(q, int(u[e])), _find(q, int(v[e]))
            if ra == rb:
                ok = False
                break
            q[ra] = rb
        if not ok:
            continue
        cost = sum(int(w[e]) * 2**32 + e for e in sub)
        if best is None or cost < best:
            best, best_set = cost, sub
    mask = np.zeros(m, np.uint8)
    mask[list(best_set)] = 1
    return mask, int(sum(int(w[e]) for e in best_set))


def by_definition(u, v, w, n):
    """e in MSF iff u_e != v_e and no path joins u_e, v_e using only edges f
    with (w_f, f) < (w_e, e).  O(m^2); meant for m up to a few thousand."""
    m = len(u)
    keys = [(int(w[e]) << 32) | e for e in range(m)]
    mask = np.zeros(m, np.uint8)
    for e in range(m):
        if u[e] == v[e]:
            continue
        adj = {}
        for f in range(m):
            if keys[f] < keys[e] and u[f] != v[f]:
                adj.setdefault(int(u[f]), []).append(int(v[f]))
                adj.setdefault(int(v[f]), []).append(int(u[f]))
        seen = {int(u[e])}
        stack = [int(u[e])]
        while stack:
            x = stack.pop()
            for y in adj.get(x, ()):
                if y not in seen:
                    seen.add(y)
                    stack.append(y)
        if int(v[e]) not in seen:
            mask[e] = 1
    return mask, int(sum(int(w[e]) for e in range(m) if mask[e]))
