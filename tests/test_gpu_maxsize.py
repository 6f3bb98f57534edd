"""The library's largest inputs on one MI355X (288 GB): edge positions above
2^31 in the (weight, position) keys and in the output mask, vertex ids up to
2^31 - 2, both algorithms.  Borůvka runs at the interface's limit of
m = 2^32 - 1 edges (44 B of workspace per edge); Filter-Borůvka, whose
workspace takes 76 B per edge, at the largest m that fits beside its input,
2^31 + 2^29 + 1.  Each case needs up to ~250 GB of device memory; nothing
else is held while it runs."""
import gc

import numpy as np
import pytest

import oracle
from gpu_util import banner, to_dev
from known_msf import known_msf_graph

pytestmark = pytest.mark.gpu

M_MAX = 2**32 - 1
M_FILTER = 2**31 + 2**29 + 1
N_MAX = 2**31 - 1
ALGOS = ("boruvka", "filter")


def _release():
    import torch
    gc.collect()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def _equal_chunks(a, b, chunk=1 << 30):
    import torch
    return all(torch.equal(a[i:i + chunk], b[i:i + chunk]) for i in range(0, a.numel(), chunk))


@pytest.mark.timeout(900)
@pytest.mark.parametrize("local", [False, True])
@pytest.mark.parametrize("algo,m", [("boruvka", M_MAX), ("filter", M_FILTER)])
def test_maximum_edge_count(algo, m, local):
    """m edges on 2^24 vertices, MSF known by construction (a light spanning
    tree scattered over all positions, equal-weight and lighter copies of a
    quarter of its edges, every other edge heavier).  local: ids rise along
    the edge list (the window kernels and the per-tile parallel-edge table
    run); else uniform random ids."""
    import torch
    import paper_2302_12199_amd as msf
    n = 1 << 24
    banner(f"maximum edge count {algo} m={m} n=2^24 local={local}: generating")
    _release()
    dev = torch.device("cuda:0")
    u, v, w, exp, total, count = known_msf_graph(m, n, device=dev, seed=31 + int(local),
                                                 local=local)
    ws = torch.empty(msf.workspace_bytes(m, n, algo=algo), dtype=torch.uint8, device=dev)
    mask = torch.full((m,), 7, dtype=torch.uint8, device=dev)
    try:
        banner(f"maximum edge count {algo} local={local}: solving")
        _, t, st = msf.compute(u, v, w, n, workspace=ws, mask_out=mask, algo=algo)
        torch.cuda.synchronize()
        assert t == total and st["total_weight"] == total
        assert st["msf_edges"] == count
        assert _equal_chunks(mask, exp)
    finally:
        del u, v, w, exp, ws, mask
        _release()


@pytest.mark.timeout(600)
def test_maximum_vertex_count():
    """n = 2^31 - 1 with 2^22 edges whose ends spread over every id, 0 and
    n - 1 included; the oracle runs on the same graph with its ids renumbered
    densely (an isomorphic graph with the same edge ids, so the same MSF)."""
    import torch
    import paper_2302_12199_amd as msf
    banner("maximum vertex count n=2^31-1 m=2^22")
    _release()
    m = 1 << 22
    rng = np.random.default_rng(41)
    u = rng.integers(0, N_MAX, m, dtype=np.int64).astype(np.int32)
    v = rng.integers(0, N_MAX, m, dtype=np.int64).astype(np.int32)
    # a few hubs so that components grow large, the extreme ids, copies
    hubs = rng.integers(0, N_MAX, 64, dtype=np.int64).astype(np.int32)
    v[::3] = hubs[rng.integers(0, 64, len(v[::3]))]
    u[:4] = [0, N_MAX - 1, N_MAX - 1, 0]
    v[:4] = [N_MAX - 1, N_MAX - 2, 0, 0]
    w = rng.integers(0, 1 << 20, m, dtype=np.uint32)
    ids, inv = np.unique(np.concatenate([u, v]), return_inverse=True)
    assert ids[0] == 0 and ids[-1] == N_MAX - 1
    rm, rt, _ = oracle.kruskal(inv[:m].astype(np.int32), inv[m:].astype(np.int32), w, len(ids))
    tu, tv, tw = to_dev(u, v, w)
    ws = torch.empty(max(msf.workspace_bytes(m, N_MAX, algo=a) for a in ALGOS),
                     dtype=torch.uint8, device=tu.device)
    try:
        for algo in ALGOS:
            banner(f"maximum vertex count: {algo}")
            mask, t, st = msf.compute(tu, tv, tw, N_MAX, workspace=ws, algo=algo)
            assert t == rt and st["msf_edges"] == int(rm.sum())
            assert np.array_equal(mask.cpu().numpy(), rm)
    finally:
        del tu, tv, tw, ws
        _release()


@pytest.mark.timeout(900)
def test_batched_maximum_sizes():
    """One batch whose edge offsets pass 2^32: a graph of 2^32 - 1 edges and
    one of 2^29 + 3 (each solved by the workgroups of one XCD together), then
    two smaller ones at offsets above 2^32 (one workgroup each, one with its
    state in LDS, one in a global slot); known MSFs, the small random graph
    against the oracle."""
    import torch
    import paper_2302_12199_amd as msf
    banner("batched maximum sizes: generating")
    _release()
    dev = torch.device("cuda:0")
    parts, exps, totals, counts, ns = [], [], [], [], []
    for m, n, seed in ((M_MAX, 1 << 20, 51), (2**29 + 3, 1 << 18, 52), (2**20 - 3, 1 << 16, 53)):
        u, v, w, exp, t, c = known_msf_graph(m, n, device=dev, seed=seed)
        parts.append((u, v, w))
        exps.append(exp)
        totals.append(t)
        counts.append(c)
        ns.append(n)
    rng = np.random.default_rng(54)
    su = rng.integers(0, 3000, 20000).astype(np.int32)
    sv = rng.integers(0, 3000, 20000).astype(np.int32)
    sw = rng.integers(0, 50, 20000).astype(np.uint32)
    rm, rt, _ = oracle.kruskal(su, sv, sw, 3000)
    parts.insert(2, tuple(to_dev(su, sv, sw)))
    exps.insert(2, torch.from_numpy(rm).to(dev))
    totals.insert(2, rt)
    ns.insert(2, 3000)
    sizes = [p[0].numel() for p in parts]
    eo = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    vo = np.concatenate([[0], np.cumsum(ns)]).astype(np.int64)
    assert eo[2] > 2**32
    cat = [torch.empty(int(eo[-1]), dtype=torch.int32, device=dev) for _ in range(3)]
    for g, p in enumerate(parts):
        for k in range(3):
            cat[k][eo[g]:eo[g + 1]] = p[k]
    del parts
    _release()
    b = None
    try:
        b = msf.Batch(cat[0], cat[1], cat[2], eo, vo)
        banner("batched maximum sizes: solving")
        b.launch()
        torch.cuda.synchronize()
        got = b.totals[:4].cpu().numpy().view(np.uint64)
        assert [int(x) for x in got] == totals
        for g in range(4):
            assert _equal_chunks(b.mask[eo[g]:eo[g + 1]], exps[g])
    finally:
        del cat, exps, b
        _release()
