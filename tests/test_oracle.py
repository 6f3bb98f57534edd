"""Pins for the CPU oracle (no GPU).  Each test ties the oracle to something
other than itself: brute force, the O(m^2) definition, closed forms, a library
routine, an independent certificate checker, or invariants from the paper."""
import numpy as np
import pytest

import graphgen
import oracle

pytestmark = pytest.mark.filterwarnings("ignore::DeprecationWarning")


def rand_multigraph(rng, n, m, wmax, loops=True):
    u = rng.integers(0, n, m).astype(np.int32)
    v = rng.integers(0, n, m).astype(np.int32)
    if not loops:
        v = np.where(u == v, (v + 1) % n, v).astype(np.int32)
    w = rng.integers(0, wmax + 1, m).astype(np.uint32)
    return u, v, w


def test_golden_hand_example(golden):
    g = golden("hand_example_7v.txt")
    mask, total, count = oracle.kruskal(g["u"], g["v"], g["w"], g["n"])
    assert (mask == g["mask"]).all()
    assert total == g["total"] and count == g["count"]
    _, _, rounds = oracle.boruvka_rounds(g["u"], g["v"], g["w"], g["n"])
    assert rounds == g["rounds"]


@pytest.mark.parametrize("wmax", [0, 1, 3, 255])
def test_kruskal_vs_brute_force(wmax):
    rng = np.random.default_rng(100 + wmax)
    for _ in range(120):
        n = int(rng.integers(1, 9))
        m = int(rng.integers(0, 14))
        u, v, w = rand_multigraph(rng, n, m, wmax)
        mask, total, count = oracle.kruskal(u, v, w, n)
        bm, bt = oracle.brute_force(u, v, w, n)
        assert (mask == bm).all(), (u, v, w)
        assert total == bt
        assert count == n - oracle.components(u, v, n)


def test_kruskal_vs_definition():
    rng = np.random.default_rng(7)
    for t in range(25):
        n = int(rng.integers(2, 40))
        m = int(rng.integers(0, 120))
        u, v, w = rand_multigraph(rng, n, m, [0, 2, 9, 2**32 - 1][t % 4])
        mask, total, _ = oracle.kruskal(u, v, w, n)
        dm, dt = oracle.by_definition(u, v, w, n)
        assert (mask == dm).all()
        assert total == dt


def test_closed_forms():
    # a forest without self-loops or duplicates: every edge is in the MSF
    u = np.array([0, 1, 1, 5, 6], np.int32)
    v = np.array([1, 2, 3, 6, 7], np.int32)
    w = np.array([9, 3, 3, 1, 2**32 - 1], np.uint32)
    mask, total, count = oracle.kruskal(u, v, w, 9)
    assert mask.all() and total == int(w.astype(np.uint64).sum()) and count == 5
    # cycle C_k: all edges but the (w, id)-maximum
    for k in (3, 4, 10):
        for wt in (np.full(k, 5), np.arange(k)[::-1] + 1, np.array([7] * (k - 1) + [1])):
            u = np.arange(k, dtype=np.int32)
            v = ((np.arange(k) + 1) % k).astype(np.int32)
            w = wt.astype(np.uint32)
            keys = (w.astype(np.uint64) << np.uint64(32)) | np.arange(k, dtype=np.uint64)
            mask, total, _ = oracle.kruskal(u, v, w, k)
            expect = np.ones(k, np.uint8)
            expect[int(np.argmax(keys))] = 0
            assert (mask == expect).all()
    # K_n with equal weights and lexicographic ids: the star at vertex 0
    n = 9
    pairs = [(i, j) for i in range(n) for j in range(i + 1, n)]
    u = np.array([p[0] for p in pairs], np.int32)
    v = np.array([p[1] for p in pairs], np.int32)
    w = np.full(len(pairs), 1000, np.uint32)
    mask, total, count = oracle.kruskal(u, v, w, n)
    assert (mask == (u == 0)).all() and total == (n - 1) * 1000
    # only self-loops: empty MSF
    mask, total, count = oracle.kruskal(np.arange(5, dtype=np.int32),
                                        np.arange(5, dtype=np.int32),
                                        np.ones(5, np.uint32), 5)
    assert not mask.any() and total == 0 and count == 0
    # a star: all its edges
    mask, total, _ = oracle.kruskal(np.zeros(6, np.int32), np.arange(1, 7, dtype=np.int32),
                                    np.array([5, 5, 1, 2**31, 0, 7], np.uint32), 7)
    assert mask.all()
    # empty inputs
    assert oracle.kruskal([], [], [], 0)[1:] == (0, 0)
    assert oracle.kruskal([], [], [], 5)[1:] == (0, 0)


def test_input_validation():
    with pytest.raises(oracle.OracleError) as e:
        oracle.kruskal([0], [3], [1], 3)
    assert e.value.status == oracle.ERANGE
    with pytest.raises(oracle.OracleError) as e:
        oracle.kruskal([0], [-1], [1], 3)
    assert e.value.status == oracle.ERANGE
    with pytest.raises(oracle.OracleError) as e:
        oracle.kruskal([0], [0], [1], 0)
    assert e.value.status == oracle.EINVAL


def test_total_vs_networkx():
    nx = pytest.importorskip("networkx")
    rng = np.random.default_rng(11)
    for wmax in (3, 255, 2**31):
        n, m = 300, 2000
        u, v, w = rand_multigraph(rng, n, m, wmax)
        _, total, count = oracle.kruskal(u, v, w, n)
        g = nx.MultiGraph()
        g.add_nodes_from(range(n))
        for a, b, c in zip(u.tolist(), v.tolist(), w.tolist()):
            g.add_edge(a, b, weight=c)
        edges = list(nx.minimum_spanning_edges(g, algorithm="kruskal", data=True, keys=True))
        assert total == sum(d["weight"] for *_, d in edges)
        assert count == len(edges)


def test_total_vs_scipy():
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import minimum_spanning_tree
    rng = np.random.default_rng(12)
    n, m = 500, 4000
    u, v, w = rand_multigraph(rng, n, m, 1000, loops=False)
    _, total, _ = oracle.kruskal(u, v, w, n)
    # scipy sums duplicate COO entries and treats 0 as "no edge": reduce
    # parallel edges to their minimum first and shift weights by +1.
    a, b = np.minimum(u, v).astype(np.int64), np.maximum(u, v).astype(np.int64)
    pair = a * n + b
    best = {}
    for p, c in zip(pair.tolist(), w.tolist()):
        best[p] = min(best.get(p, c), c)
    keys = np.array(list(best.keys()), np.int64)
    vals = np.array(list(best.values()), np.float64) + 1.0
    g = coo_matrix((vals, (keys // n, keys % n)), shape=(n, n)).tocsr()
    t = minimum_spanning_tree(g)
    nedges = t.nnz
    assert int(round(t.sum())) - nedges == total


@pytest.mark.parametrize("kind", ["gnm", "rmat", "grid", "rgg", "rgg3d", "rhg"])
def test_certificate_checker_agrees(kind):
    if kind == "gnm":
        u, v, w = graphgen.gnm(4096, 40000, 1, 50, seed=3)
        n = 4096
    elif kind == "rmat":
        u, v, w = graphgen.rmat(13, 60000, wlo=1, whi=255, seed=4)
        n = 1 << 13
    elif kind == "grid":
        u, v, w = graphgen.grid(64, 80, 0.8, 0, 7, 7, seed=5)
        n = 64 * 80
    elif kind == "rgg3d":
        n = 6000
        u, v, w = graphgen.rgg3d(n, graphgen.rgg3d_radius(n, 16), 1, 254, seed=6)
    elif kind == "rhg":
        n = 6000
        u, v, w = graphgen.rhg(n, 16.0, 1, 254, seed=6)
    else:
        n = 5000
        u, v, w = graphgen.rgg2d(n, graphgen.rgg_radius(n, 8), 1e6, seed=6)
    mask, total, count = oracle.kruskal(u, v, w, n)
    rc, ct, cc = oracle.check(u, v, w, n, mask)
    assert rc == 0 and ct == total and cc == count


def test_certificate_checker_rejects_wrong_forests():
    u, v, w = graphgen.gnm(2000, 12000, 1, 100, seed=8)
    n = 2000
    mask, _, _ = oracle.kruskal(u, v, w, n)
    msf = np.nonzero(mask)[0]
    non = np.nonzero((mask == 0) & (u != v))[0]
    m2 = mask.copy(); m2[msf[5]] = 0
    assert oracle.check(u, v, w, n, m2)[0] == 3          # too few edges
    m2 = mask.copy(); m2[non[0]] = 1
    assert oracle.check(u, v, w, n, m2)[0] == 2           # closes a cycle
    # a self-loop marked in F (the graph gets one appended)
    uu, vv, ww = (np.append(u, 17).astype(np.int32), np.append(v, 17).astype(np.int32),
                  np.append(w, 1).astype(np.uint32))
    m3 = np.append(mask, 1).astype(np.uint8)
    assert oracle.check(uu, vv, ww, n, m3)[0] == 1
    assert oracle.check(uu, vv, ww, n, np.append(mask, 0).astype(np.uint8))[0] == 0
    # swap: drop an MSF edge and add a heavier edge reconnecting the two trees
    rng = np.random.default_rng(0)
    found = False
    for e in rng.permutation(msf)[:200]:
        m2 = mask.copy(); m2[e] = 0
        # vertices on u[e]'s side after removing e
        adj = {}
        for f in np.nonzero(m2)[0]:
            adj.setdefault(int(u[f]), []).append(int(v[f]))
            adj.setdefault(int(v[f]), []).append(int(u[f]))
        side, stack = {int(u[e])}, [int(u[e])]
        while stack:
            x = stack.pop()
            for y in adj.get(x, ()):
                if y not in side:
                    side.add(y); stack.append(y)
        cross = [f for f in non if (int(u[f]) in side) != (int(v[f]) in side)]
        if cross:
            m2[cross[0]] = 1
            assert oracle.check(u, v, w, n, m2)[0] == 5
            found = True
            break
    assert found


def test_boruvka_rounds_invariants():
    for (u, v, w), n in [(graphgen.gnm(3000, 30000, 1, 2**31 - 1, seed=1), 3000),
                         (graphgen.rmat(12, 50000, wlo=1, whi=255, seed=2), 4096),
                         (graphgen.grid(50, 60, 0.8, 0, 1000000, 1000000, seed=3), 3000)]:
        mask, total, rounds = oracle.boruvka_rounds(u, v, w, n)
        km, kt, kc = oracle.kruskal(u, v, w, n)
        assert (mask == km).all() and total == kt
        assert sum(r["found"] for r in rounds) == kc
        # |V'| <= |V|/2 per round (Sec. II-C) and at most log2(n) rounds
        for a, b in zip(rounds, rounds[1:]):
            assert b["live"] <= a["live"] // 2
        assert len(rounds) <= int(np.ceil(np.log2(n)))


def test_metamorphic():
    rng = np.random.default_rng(5)
    u, v, w = rand_multigraph(rng, 200, 1500, 40)
    n = 200
    mask, total, _ = oracle.kruskal(u, v, w, n)
    # strictly increasing weight map
    m2, _, _ = oracle.kruskal(u, v, (2 * w + 1).astype(np.uint32), n)
    assert (m2 == mask).all()
    # vertex permutation
    p = rng.permutation(n).astype(np.int32)
    m2, t2, _ = oracle.kruskal(p[u], p[v], w, n)
    assert (m2 == mask).all() and t2 == total
    # appended equal-weight copies (larger ids) and self-loops change nothing
    uu = np.concatenate([u, u[:300], np.arange(50, dtype=np.int32)])
    vv = np.concatenate([v, v[:300], np.arange(50, dtype=np.int32)])
    ww = np.concatenate([w, w[:300], np.zeros(50, np.uint32)])
    m2, t2, _ = oracle.kruskal(uu, vv, ww, n)
    assert (m2[:len(u)] == mask).all() and not m2[len(u):].any() and t2 == total


def test_sort_step_matches_library_sort():
    rng = np.random.default_rng(3)
    for k in (0, 1, 17, 100000):
        a = rng.integers(0, 2**63, k, dtype=np.uint64) * np.uint64(2) + rng.integers(0, 2, k).astype(np.uint64)
        assert (oracle.sort_u64(a) == np.sort(a)).all()


def test_filter_reference_matches_kruskal_for_any_quantile():
    # Filter-Kruskal-style filtering is exact for every pivot (Sec. V)
    u, v, w = graphgen.rmat(11, 40000, wlo=1, whi=2**31 - 1, seed=21)
    n = 1 << 11
    km, kt, _ = oracle.kruskal(u, v, w, n)
    for q in (0.0, 1.0 / 40000, 0.01, 0.5, 0.99, 1.0):
        mask, total, trace = oracle.filter_boruvka(u, v, w, n, seed=3, sample=512, q=q,
                                                   min_split=500)
        assert (mask == km).all() and total == kt
        if 0.0 < q < 1.0:
            assert len(trace) > 0
        for t in trace:
            assert 0 <= t["light"] <= t["edges"] and t["kept"] <= t["edges"] - t["light"]


def test_filter_reference_pivot_is_sample_quantile():
    from oracle.filter_ref import pivot_index, sample_positions
    pos = sample_positions(7, 0, 1000, 4096)
    assert pos.min() >= 0 and pos.max() < 1000
    # 4096 draws over 1000 positions: every position is hit about 4 times
    assert len(np.unique(pos)) > 950
    assert pivot_index(0.5, 4096) == 2047 and pivot_index(0.0, 4096) == 0
    assert pivot_index(1.0, 4096) == 4095


def test_mlp_reference_gradient_matches_finite_differences():
    from oracle import mlp_ref
    rng = np.random.default_rng(3)
    p = mlp_ref.init_params(1)
    x = rng.normal(0, 1, (7, mlp_ref.IN))
    t = rng.normal(0, 1, 7)
    loss, g = mlp_ref.loss_and_grad(p, x, t)
    eps = 1e-6
    idx = rng.choice(mlp_ref.P, 80, replace=False)
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += eps
        pm[i] -= eps
        fd = (mlp_ref.loss_and_grad(pp, x, t)[0] - mlp_ref.loss_and_grad(pm, x, t)[0]) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-6 + 1e-5 * abs(fd)


def test_mlp_reference_bf16_rounding():
    from oracle import mlp_ref
    vals = np.array([1.0, 1.0 + 2**-8, 1.0 + 2**-7 + 2**-9, -3.14159, 0.0, 1e-40], np.float32)
    r = mlp_ref.bf16(vals)
    assert r[0] == 1.0 and r[1] == 1.0            # tie -> even
    assert r[2] == 1.0 + 2**-7                    # below half a step -> down
    assert mlp_ref.bf16(np.float32(1.0 + 2**-7 + 2**-8))[()] == 1.0 + 2**-6   # tie -> even (up)
    assert abs(r[3] + 3.140625) < 1e-12
    # every result is representable in bfloat16
    bits = r.astype(np.float32).view(np.uint32)
    assert (bits & 0xFFFF == 0).all()
