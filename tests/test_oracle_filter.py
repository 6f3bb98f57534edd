"""Pins of the Filter-Borůvka parts of the oracle (no GPU): the pivot
sampler's generator, the pivot-network features, and the per-split trace,
each against something other than the code under test -- a published
generator output, a hand-worked example, closed forms and library routines,
and a second formulation of the trace from set definitions."""
import math
import os
import statistics
from fractions import Fraction

import numpy as np
import pytest
from scipy.sparse import coo_matrix
from scipy.sparse.csgraph import connected_components

import graphgen
import oracle
from oracle import features, mlp_ref
from oracle.filter_def import trace_by_definition
from oracle.filter_ref import GAMMA, MASK64, _mix, filter_boruvka, pivot_index, sample_positions

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_pivot_stream_mix_is_published_splitmix64():
    # SplitMix64 (Steele, Lea & Flood 2014) seeded with 0: its first four outputs
    # are the widely published reference sequence.
    want = [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F, 0xF88BB8A8724C81EC]
    assert [_mix((i * GAMMA) & MASK64) for i in range(1, 5)] == want


def test_sample_positions_map_the_stream_to_positions():
    # position = floor(r * len / 2^64) with r the stream output: bounds and the
    # extreme lengths
    for k in (1, 2, 3, 1000, 2**31 - 1, 2**32 - 1):
        pos = sample_positions(11, 3, k, 300)
        assert pos.min() >= 0 and pos.max() < k
    assert (sample_positions(11, 3, 1, 50) == 0).all()
    base = _mix(_mix(11) ^ (0x50495654 + 3))
    r0 = _mix((base + GAMMA) & MASK64)
    assert sample_positions(11, 3, 1000, 1)[0] == (r0 * 1000) >> 64


def _golden_features():
    d = {}
    for line in open(os.path.join(ROOT, "tests", "golden", "pivot_features_example.txt")):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        k, _, rest = line.partition(" ")
        d[k] = rest.split()
    return d


def test_features_hand_example():
    d = _golden_features()
    got = features.pivot_features([int(x) for x in d["weights"]], [int(x) for x in d["ends"]],
                                  int(d["comps"][0]), int(d["edges"][0]), int(d["depth"][0]))
    want = [float(Fraction(x)) for x in d["features"]]
    assert len(want) == 16
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-15)


def test_features_closed_forms():
    # all weights equal: every weight statistic is L(w0), no spread, all ties
    f = features.pivot_features([1000] * 64, list(range(128)), 10, 500, 0)
    L = math.log2(1001) / 32
    assert np.allclose(f[[0, 1, 2, 3, 4, 5, 8, 9]], L, atol=1e-15)
    assert f[6] == 0 and f[7] == 1 and f[14] == 0 and f[15] == 1
    # a single draw: no ties by definition; its two ends repeat iff a self-loop
    f1 = features.pivot_features([7], [3, 3], 1, 1, 2)
    assert f1[7] == 0 and f1[6] == 0 and f1[14] == 1 and f1[13] == 2 / 16
    assert features.pivot_features([7], [3, 4], 1, 1, 2)[14] == 0
    # a star: every drawn edge has end 0, so of 2k ends k are 0 (k - 1 repeats)
    # plus k distinct leaves
    k = 100
    ends = []
    for i in range(k):
        ends += [0, i + 1]
    assert features.pivot_features(list(range(1, k + 1)), ends, 5, 9, 1)[14] == (k - 1) / (2 * k - 1)


@pytest.mark.parametrize("s", [100, 4096, 8192])
def test_features_against_library_statistics(s):
    rng = np.random.default_rng(s)
    w = rng.integers(0, 2**32, s, dtype=np.uint64)
    w[: s // 5] = 77                                   # force ties
    ends = rng.integers(0, 500, 2 * min(s, 2048))
    f = features.pivot_features(w, ends, 1234, 10**6, 3)
    L = np.sort(np.log2(1.0 + w.astype(np.float64)) / 32)
    for j, q in enumerate(features.QUANTILES):
        # for these sizes q * (s - 1) is nowhere near an integer, so the single
        # precision index equals numpy's 'lower' quantile
        assert f[j] == np.quantile(L, q, method="lower")
    assert math.isclose(f[5], statistics.fmean(L.tolist()), rel_tol=1e-13)
    assert math.isclose(f[6], statistics.pstdev(L.tolist()), rel_tol=1e-12)
    assert f[7] == (s - len(np.unique(w))) / (s - 1)
    assert f[14] == (len(ends) - len(np.unique(ends))) / (len(ends) - 1)
    assert f[8] == L[0] and f[9] == L[-1]


def test_quantile_index_is_taken_in_single_precision():
    assert features.quantile_index(0.5, 4096) == 2047
    assert features.quantile_index(0.9, 8) == 6              # 0.9f * 7 = 6.2999997
    assert features.quantile_index(0.1, 11) == 1             # 0.1f * 10 = 1.0000000149 -> 1.0f
    # 0.7f is 0.699999988: its exact product with 10 lies below 7 (floor 6),
    # but the product rounded to single precision is 7.0f, as on the device
    assert float(np.float32(0.7)) * 10 < 7
    assert features.quantile_index(0.7, 11) == 7


def _graphs():
    yield "gnm", graphgen.gnm(3000, 60000, 1, 2**31 - 1, seed=3), 3000
    yield "rmat_w255", graphgen.rmat(12, 70000, seed=4, wlo=1, whi=255), 4096
    yield "gnm_w3_loops", _with_loops(*graphgen.gnm(3000, 50000, 1, 3, seed=5)), 3000


def _with_loops(u, v, w):
    u = np.concatenate([u, np.arange(300, dtype=np.int32)])
    v = np.concatenate([v, np.arange(300, dtype=np.int32)])
    w = np.concatenate([w, np.full(300, 2, np.uint32)])
    return u, v, w


@pytest.mark.parametrize("q", [0.0, 0.05, 0.5, 0.9, 1.0])
@pytest.mark.parametrize("sample", [1, 100, 777])
def test_filter_trace_equals_its_definition(q, sample):
    """filter_ref's union-find recursion against the set definitions: every
    split's edge count, pivot, light count, kept count and features."""
    for name, (u, v, w), n in _graphs():
        mask, total, tr = filter_boruvka(u, v, w, n, seed=7, sample=sample, q=q, min_split=2000)
        td = trace_by_definition(u, v, w, n, seed=7, sample=sample, q=q, min_split=2000)
        assert len(tr) == len(td), name
        for i, (a, b) in enumerate(zip(tr, td)):
            for k in ("edges", "pivot", "light", "kept"):
                assert a[k] == b[k], (name, i, k)
            np.testing.assert_array_equal(a["features"], b["features"])
        km, kt, _ = oracle.kruskal(u, v, w, n)
        assert (mask == km).all() and total == kt


def test_top_split_kept_by_connected_components():
    """kept of the first split = heavy edges whose ends lie in different
    connected components of the light edges (the light MSF has the light
    edges' components), counted with a library routine."""
    for name, (u, v, w), n in _graphs():
        _, _, tr = filter_boruvka(u, v, w, n, seed=9, sample=512, q=0.3, min_split=2000)
        keys = (w.astype(np.uint64) << np.uint64(32)) | np.arange(len(u), dtype=np.uint64)
        light = keys <= np.uint64(tr[0]["pivot"])
        g = coo_matrix((np.ones(int(light.sum())), (u[light], v[light])), shape=(n, n))
        _, lab = connected_components(g, directed=False)
        heavy = ~light
        kept = int((lab[u[heavy]] != lab[v[heavy]]).sum())
        assert tr[0]["light"] == int(light.sum())
        assert tr[0]["kept"] == kept, name
        # the pivot is an order statistic of the drawn keys
        pos = sample_positions(9, 0, len(u), 512)
        assert tr[0]["pivot"] == int(np.sort(keys[pos])[pivot_index(0.3, 512)])


def test_network_quantile_closed_forms():
    assert mlp_ref.quantile(0.0) == 0.5
    assert mlp_ref.quantile(math.log(3.0)) == pytest.approx(0.75, rel=1e-15)
    z = np.linspace(-5, 5, 21)
    np.testing.assert_allclose(mlp_ref.quantile(z) + mlp_ref.quantile(-z), 1.0, atol=1e-15)
    assert mlp_ref.quantile(-50.0) == 2.0**-10 and mlp_ref.quantile(50.0) == 1 - 2.0**-10
    assert mlp_ref.quantile(math.log(2.0**-10 / (1 - 2.0**-10))) == pytest.approx(2.0**-10)


def test_network_forward_hand_example():
    """A network wired by hand: hidden unit 0 of layer 1 is relu(2 x0 - x1 + 1),
    unit 0 of layer 2 copies it, the output is 3 * that - 0.5; every other
    weight is zero.  Worked out: x = (1, 4): relu(2 - 4 + 1) = 0 -> z = -0.5;
    x = (3, 1): relu(6 - 1 + 1) = 6 -> z = 17.5."""
    d = {k: np.zeros(s) for k, s in mlp_ref.SIZES}
    d["W1"][0, 0], d["W1"][0, 1], d["b1"][0] = 2.0, -1.0, 1.0
    d["W2"][0, 0] = 1.0
    d["w3"][0], d["b3"][0] = 3.0, -0.5
    p = mlp_ref.pack(d)
    x = np.zeros((2, 16))
    x[0, :2] = (1, 4)
    x[1, :2] = (3, 1)
    z, _ = mlp_ref.forward(p, x)
    assert z.tolist() == [-0.5, 17.5]
    # bfloat16 rounding leaves these exactly representable values alone
    assert mlp_ref.forward(p, x, bf=True)[0].tolist() == [-0.5, 17.5]
    # the magnitude pass: |2 x0| + |x1| + 1 for both samples, times 3, plus 0.5
    assert mlp_ref.magnitude(p, x).tolist() == [3 * (2 + 4 + 1) + 0.5, 3 * (6 + 1 + 1) + 0.5]


def test_stream_of_a_redraw():
    from oracle.filter_ref import stream_base
    first = _mix(_mix(5) ^ (0x50495654 + 2))
    assert stream_base(5, 2) == first == stream_base(5, 2, 0)
    assert stream_base(5, 2, 3) == _mix((first + 3 * GAMMA) & MASK64)
    assert len({stream_base(5, 2, a) for a in range(6)}) == 6


def test_balanced_band_is_the_papers_third_for_the_median():
    from oracle.filter_ref import balanced
    assert balanced(100, 300, 0.5) and balanced(200, 300, 0.5)
    assert not balanced(99, 300, 0.5) and not balanced(201, 300, 0.5)
    assert balanced(0, 100, 0.1) and not balanced(30, 100, 0.1)


@pytest.mark.parametrize("q", [0.5, 0.2])
def test_balanced_retry(q):
    """One-edge samples often split badly; with redraws every split that did
    not use up its draws lies in the band, and the MSF is unchanged."""
    from oracle.filter_ref import balanced
    u, v, w = graphgen.gnm(3000, 90000, 1, 2**31 - 1, seed=12)
    km, kt, _ = oracle.kruskal(u, v, w, 3000)
    _, _, plain = filter_boruvka(u, v, w, 3000, seed=4, sample=1, q=q, min_split=1500)
    info = {}
    mask, total, tr = filter_boruvka(u, v, w, 3000, seed=4, sample=1, q=q, min_split=1500,
                                     retries=6, info=info)
    assert (mask == km).all() and total == kt
    assert info["retries"] > 0 and sum(t["attempts"] - 1 for t in tr) == info["retries"]
    for t in tr:
        assert 1 <= t["attempts"] <= 7
        if t["attempts"] < 7:
            assert balanced(t["light"], t["edges"], q)
    # without redraws the one-edge pivots leave unbalanced splits
    assert any(not balanced(t["light"], t["edges"], q) for t in plain)
    assert all(t["attempts"] == 1 for t in plain)


@pytest.mark.parametrize("defer", [0, 200, 3000, 10**6])
def test_deferral_keeps_the_msf(defer):
    """Handing small filtered sets back a level changes the work, never the
    MSF.  On this graph the second split's 2719 filtered edges go back to the
    top level below 3000, which then filters them with its heavy edges."""
    u, v, w = graphgen.rmat(13, 150000, wlo=1, whi=2**31 - 1, seed=13)
    n = 1 << 13
    km, kt, _ = oracle.kruskal(u, v, w, n)
    base_info, info = {}, {}
    _, _, plain = filter_boruvka(u, v, w, n, seed=2, sample=256, q=0.3, min_split=1000,
                                 info=base_info)
    mask, total, tr = filter_boruvka(u, v, w, n, seed=2, sample=256, q=0.3, min_split=1000,
                                     defer=defer, info=info)
    assert (mask == km).all() and total == kt
    if defer < plain[1]["kept"] + 1:
        assert info["deferrals"] == 0 and len(tr) == len(plain)
        for a, b in zip(tr, plain):
            assert {k: x for k, x in a.items() if k != "features"} == \
                {k: x for k, x in b.items() if k != "features"}
    else:
        assert info["deferrals"] > 0
        assert tr[0]["deferred_in"] == plain[1]["kept"]
    # a split's handed-back edges came from a set below the threshold
    assert all(t["deferred_in"] < max(defer, 1) for t in tr)
