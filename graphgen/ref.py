"""numpy restatement of graphgen.c, used only to pin the C generators.

Same definitions, written independently with numpy uint64 arithmetic
(wrap-around multiplication matches C's unsigned semantics).
"""
from __future__ import annotations

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
M1 = np.uint64(0xBF58476D1CE4E5B9)
M2 = np.uint64(0x94D049BB133111EB)
TAG_GNM, TAG_RMAT, TAG_PERM, TAG_RMAT_W, TAG_GRID_KEEP, TAG_GRID_W, TAG_RGG = 1, 2, 3, 4, 5, 6, 7


def mix(z):
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * M1
        z = (z ^ (z >> np.uint64(27))) * M2
    return z ^ (z >> np.uint64(31))


def base(seed: int, tag: int):
    return mix(mix(np.uint64(seed)) ^ np.uint64(tag))


def draw(b, k):
    k = np.asarray(k, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return mix(np.uint64(b) + (k + np.uint64(1)) * GAMMA)


def below(r, n: int):
    r = np.asarray(r, dtype=np.uint64)
    n = np.uint64(n)
    hi, lo = r >> np.uint64(32), r & np.uint64(0xFFFFFFFF)
    with np.errstate(over="ignore"):
        return (hi * n + ((lo * n) >> np.uint64(32))) >> np.uint64(32)


def gnm(n, m, wlo, whi, seed):
    b = base(seed, TAG_GNM)
    i = np.arange(m, dtype=np.uint64)
    a = below(draw(b, 3 * i), n)
    d = below(draw(b, 3 * i + 1), n - 1)
    v = (a + np.uint64(1) + d) % np.uint64(n)
    w = np.uint64(wlo) + below(draw(b, 3 * i + 2), whi - wlo + 1)
    return a.astype(np.int32), v.astype(np.int32), w.astype(np.uint32)


def _feistel(x, scale, keys):
    h = (scale + 1) // 2
    mask, lim = np.uint64((1 << h) - 1), np.uint64(1 << scale)
    x = np.asarray(x, dtype=np.uint64).copy()
    todo = np.ones(len(x), bool)
    while todo.any():
        L, R = x[todo] >> np.uint64(h), x[todo] & mask
        for k in keys:
            F = mix(R ^ k) & mask
            L, R = R, L ^ F
        y = (L << np.uint64(h)) | R
        x[todo] = y
        idx = np.nonzero(todo)[0]
        todo[idx[y < lim]] = False
    return x


def rmat(scale, m, a, b, c, wlo, whi, permute, seed):
    ta = np.uint64(int(np.floor(a * 4294967296.0)))
    tab = np.uint64(int(np.floor((a + b) * 4294967296.0)))
    tabc = np.uint64(int(min(np.floor((a + b + c) * 4294967296.0), 4294967295.0)))
    bb, bw = base(seed, TAG_RMAT), base(seed, TAG_RMAT_W)
    per = (scale + 1) // 2
    i = np.arange(m, dtype=np.uint64)
    u = np.zeros(m, np.uint64)
    v = np.zeros(m, np.uint64)
    for lvl in range(scale):
        r = draw(bb, i * np.uint64(per) + np.uint64(lvl >> 1))
        x = (r & np.uint64(0xFFFFFFFF)) if lvl & 1 else (r >> np.uint64(32))
        ub = (x >= tab).astype(np.uint64)
        vb = (((x >= ta) & (x < tab)) | (x >= tabc)).astype(np.uint64)
        u = (u << np.uint64(1)) | ub
        v = (v << np.uint64(1)) | vb
    if permute:
        bp = base(seed, TAG_PERM)
        keys = [draw(bp, k) for k in range(4)]
        u, v = _feistel(u, scale, keys), _feistel(v, scale, keys)
    w = np.uint64(wlo) + below(draw(bw, i), whi - wlo + 1)
    return u.astype(np.int32), v.astype(np.int32), w.astype(np.uint32)


def grid(rows, cols, keep, wmode, wlo, whi, seed):
    thr = 0xFFFFFFFF if keep >= 1.0 else int(np.floor(keep * 4294967296.0))
    bk, bw = base(seed, TAG_GRID_KEEP), base(seed, TAG_GRID_W)
    us, vs, cs = [], [], []
    c = 0
    for i in range(rows):
        for j in range(cols):
            x = i * cols + j
            if j + 1 < cols:
                us.append(x); vs.append(x + 1); cs.append(c); c += 1
            if i + 1 < rows:
                us.append(x); vs.append(x + cols); cs.append(c); c += 1
    cs = np.array(cs, dtype=np.uint64)
    keepm = (draw(bk, cs) >> np.uint64(32)) < np.uint64(thr)
    u = np.array(us, np.int64)[keepm]
    v = np.array(vs, np.int64)[keepm]
    if wmode == 0:
        w = np.full(len(u), wlo, np.uint64)
    else:
        w = np.uint64(wlo) + below(draw(bw, cs[keepm]), whi - wlo + 1)
    return u.astype(np.int32), v.astype(np.int32), w.astype(np.uint32)


def rgg2d_bruteforce(n, r, wscale, seed):
    """All-pairs RGG in the generator's id order (for small n only)."""
    b = base(seed, TAG_RGG)
    t = np.arange(n, dtype=np.uint64)
    x = (draw(b, 2 * t) >> np.uint64(11)).astype(np.float64) * 2.0**-53
    y = (draw(b, 2 * t + 1) >> np.uint64(11)).astype(np.float64) * 2.0**-53
    G = max(1, int(np.floor(1.0 / r)))
    cx = np.minimum((x * G).astype(np.int64), G - 1)
    cy = np.minimum((y * G).astype(np.int64), G - 1)
    order = np.lexsort((np.arange(n), cy * G + cx))
    x, y = x[order], y[order]
    us, vs, ws = [], [], []
    for i in range(n):
        dx, dy = x[i + 1:] - x[i], y[i + 1:] - y[i]
        d2 = dx * dx + dy * dy
        js = np.nonzero(d2 < r * r)[0]
        for j in js:
            us.append(i); vs.append(i + 1 + j)
            ws.append(int(np.floor(wscale * np.sqrt(d2[j]) + 0.5)))
    return (np.array(us, np.int32), np.array(vs, np.int32), np.array(ws, np.uint32))


TAG_RGG3, TAG_RGG3_W, TAG_RHG, TAG_RHG_W = 9, 10, 11, 12


def _edge_weights(seed, tag, m, wlo, whi):
    bw = base(seed, tag)
    return (np.uint64(wlo) + below(draw(bw, np.arange(m, dtype=np.uint64)),
                                   whi - wlo + 1)).astype(np.uint32)


def rgg3d_bruteforce(n, r, wlo, whi, seed):
    """All-pairs 3D RGG in the generator's id order (for small n only)."""
    b = base(seed, TAG_RGG3)
    t = np.arange(n, dtype=np.uint64)
    x = (draw(b, 3 * t) >> np.uint64(11)).astype(np.float64) * 2.0**-53
    y = (draw(b, 3 * t + 1) >> np.uint64(11)).astype(np.float64) * 2.0**-53
    z = (draw(b, 3 * t + 2) >> np.uint64(11)).astype(np.float64) * 2.0**-53
    G = min(max(1, int(np.floor(1.0 / r))), 1 << 10)
    c = [np.minimum((a * G).astype(np.int64), G - 1) for a in (x, y, z)]
    order = np.lexsort((np.arange(n), (c[2] * G + c[1]) * G + c[0]))
    x, y, z = x[order], y[order], z[order]
    us, vs = [], []
    for i in range(n):
        dx, dy, dz = x[i + 1:] - x[i], y[i + 1:] - y[i], z[i + 1:] - z[i]
        js = np.nonzero(dx * dx + dy * dy + dz * dz < r * r)[0]
        us += [i] * len(js)
        vs += (i + 1 + js).tolist()
    return (np.array(us, np.int32), np.array(vs, np.int32),
            _edge_weights(seed, TAG_RGG3_W, len(us), wlo, whi))


def rhg_bruteforce(n, avg_deg, wlo, whi, seed):
    """All-pairs random hyperbolic graph (threshold model, alpha = 1) in the
    generator's id order (for small n only).  Per-point values use the
    platform's libm through the math module, the adjacency test plain
    double arithmetic in the generator's order."""
    import math
    R = 2.0 * math.log(8.0 * n / (math.pi * avg_deg))
    coshR = math.cosh(R)
    b = base(seed, TAG_RHG)
    t = np.arange(n, dtype=np.uint64)
    u = (draw(b, 2 * t) >> np.uint64(11)).astype(np.float64) * 2.0**-53
    phi = (draw(b, 2 * t + 1) >> np.uint64(11)).astype(np.float64) * 2.0**-53
    order = np.lexsort((np.arange(n), phi))
    A = 1.0 + u[order] * (coshR - 1.0)
    phi = phi[order]
    B = np.sqrt(A * A - 1.0)
    C = np.array([math.cos(2.0 * math.pi * p) for p in phi.tolist()])
    S = np.array([math.sin(2.0 * math.pi * p) for p in phi.tolist()])
    us, vs = [], []
    for i in range(n):
        j = np.arange(i + 1, n)
        adj = A[i] * A[j] - B[i] * B[j] * (C[i] * C[j] + S[i] * S[j]) < coshR
        js = j[adj]
        us += [i] * len(js)
        vs += js.tolist()
    return (np.array(us, np.int32), np.array(vs, np.int32),
            _edge_weights(seed, TAG_RHG_W, len(us), wlo, whi))
