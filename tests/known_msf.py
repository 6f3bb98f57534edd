"""Graphs of any size whose minimum spanning forest is known by construction
(test infrastructure, shared by a CPU test that pins it to the oracle and the
GPU tests at the library's maximum sizes).

Every edge position holds a heavy edge (weight >= LIGHT) except the edges of
a spanning tree T (weights < LIGHT), scattered over the positions, and copies
of every fourth tree edge at other positions (ends swapped; half of them with
the same weight, half one lighter where the weight allows).  Paper Sec. II-B:
an edge that is the heaviest on some cycle under the (weight, id) order is in
no MSF.  Each heavy edge closes a cycle with T on which it is the heaviest,
and of the copies of one vertex pair all but the lightest (weight, id) are, so
the MSF is T with each tree edge at its winning copy, whatever the draws.
"""
import math

import torch

LIGHT = 1001
STRIDE = 2654435761   # tree edge k sits at position k * STRIDE mod m


def known_msf_graph(m, n, *, device, seed, local=False, chunk=1 << 27):
    """Returns (u, v, w, expected_mask, total, count): int32 tensors u, v, w
    (w holds values below 2^31, so its int32 view is the uint32 weight), the
    uint8 MSF mask, its total weight and edge count.

    local=False: heavy edges join uniform random ids; T is a random recursive
    tree (vertex k hangs below a uniform vertex of [0, k)).
    local=True: position e's heavy edge starts at id floor(e n / m) and ends
    1..4096 ids further on (mod n), so ids rise along the edge list; T is the
    path 0-1-...-(n-1)."""
    if n < 2 or m < 2 * n or math.gcd(STRIDE, m) != 1:
        raise ValueError("need n >= 2, m >= 2 n and gcd(STRIDE, m) == 1")
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    i32, i64 = torch.int32, torch.int64
    u = torch.empty(m, dtype=i32, device=device)
    v = torch.empty(m, dtype=i32, device=device)
    w = torch.empty(m, dtype=i32, device=device)
    for c0 in range(0, m, chunk):
        c1 = min(m, c0 + chunk)
        k = c1 - c0
        if local:
            a = torch.arange(c0, c1, dtype=i64, device=device) * n // m
            off = torch.randint(1, 4097, (k,), dtype=i64, device=device, generator=g)
            u[c0:c1] = a.to(i32)
            v[c0:c1] = ((a + off) % n).to(i32)
            del a, off
        else:
            u[c0:c1] = torch.randint(0, n, (k,), dtype=i32, device=device, generator=g)
            v[c0:c1] = torch.randint(0, n, (k,), dtype=i32, device=device, generator=g)
        w[c0:c1] = torch.randint(LIGHT, 2**31 - 1, (k,), dtype=i32, device=device, generator=g)

    k = torch.arange(1, n, dtype=i64, device=device)          # tree edge k joins k, par[k]
    if local:
        par = k - 1
    else:
        r = torch.rand(n - 1, dtype=torch.float64, device=device, generator=g)
        par = torch.minimum((r * k.to(torch.float64)).to(i64), k - 1)
    wt = torch.randint(0, LIGHT, (n - 1,), dtype=i64, device=device, generator=g)
    swap = torch.rand(n - 1, device=device, generator=g) < 0.5
    a = torch.where(swap, par, k)
    b = torch.where(swap, k, par)
    pos = (k * STRIDE) % m
    u[pos], v[pos], w[pos] = a.to(i32), b.to(i32), wt.to(i32)

    sel = k % 4 == 0                                           # copies, at (k + n) * STRIDE
    ks, ws, ps = k[sel], wt[sel], pos[sel]
    q = ((ks + n) * STRIDE) % m
    cw = torch.where(ks % 8 == 4, (ws - 1).clamp(min=0), ws)
    u[q], v[q], w[q] = b[sel].to(i32), a[sel].to(i32), cw.to(i32)

    exp = torch.zeros(m, dtype=torch.uint8, device=device)
    exp[pos] = 1
    copy_wins = (cw < ws) | ((cw == ws) & (q < ps))
    exp[ps[copy_wins]] = 0
    exp[q[copy_wins]] = 1
    eff = wt.clone()
    eff[sel] = torch.where(copy_wins, cw, ws)
    return u, v, w, exp, int(eff.sum().item()), n - 1
