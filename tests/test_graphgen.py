"""The seeded generators: C implementation vs the numpy restatement, plus the
statistical shape of each family (no GPU)."""
import numpy as np
import pytest

import graphgen
import graphgen.ref as ref


def same(a, b):
    return all(x.dtype == y.dtype and (x == y).all() for x, y in zip(a, b))


def test_draw_stream_matches_reference():
    for seed, tag in [(0, 1), (1, 2), (2**64 - 1, 7)]:
        for k in (0, 1, 12345, 2**40):
            assert graphgen.draw(seed, tag, k) == int(ref.draw(ref.base(seed, tag), k))


def test_splitmix_known_value():
    # SplitMix64 seeded with 0: first output 0xE220A8397B1DCDAF (Steele et al. 2014,
    # the widely published reference sequence).
    assert int(ref.mix(np.uint64(0x9E3779B97F4A7C15))) == 0xE220A8397B1DCDAF


@pytest.mark.parametrize("args", [(1000, 5000, 1, 2**31 - 1, 7), (2, 100, 5, 5, 3),
                                  (65536, 300000, 1, 255, 1)])
def test_gnm_bitexact(args):
    assert same(graphgen.gnm(*args), ref.gnm(*args))


@pytest.mark.parametrize("scale", [1, 5, 10, 11, 16])
def test_rmat_bitexact(scale):
    a = graphgen.rmat(scale, 20000, seed=9)
    b = ref.rmat(scale, 20000, .57, .19, .19, 1, 255, True, 9)
    assert same(a, b)


def test_grid_bitexact():
    assert same(graphgen.grid(37, 53, 0.8, 1, 1, 255, seed=3), ref.grid(37, 53, 0.8, 1, 1, 255, 3))
    assert same(graphgen.grid(20, 1, 1.0, 0, 9, 9, seed=1), ref.grid(20, 1, 1.0, 0, 9, 9, 1))


def test_rgg_matches_bruteforce():
    a = graphgen.rgg2d(3000, 0.03, 1e6, seed=4)
    b = ref.rgg2d_bruteforce(3000, 0.03, 1e6, 4)
    assert same(a, b)


@pytest.mark.parametrize("n,seed,deg", [(2000, 7, 12.0), (3001, 1, 16.0), (257, 3, 30.0)])
def test_rgg3d_matches_bruteforce(n, seed, deg):
    r = graphgen.rgg3d_radius(n, deg)
    assert same(graphgen.rgg3d(n, r, 1, 254, seed), ref.rgg3d_bruteforce(n, r, 1, 254, seed))


@pytest.mark.parametrize("n,seed,deg", [(2000, 8, 16.0), (3001, 2, 10.0), (400, 5, 40.0)])
def test_rhg_matches_bruteforce(n, seed, deg):
    assert same(graphgen.rhg(n, deg, 1, 254, seed), ref.rhg_bruteforce(n, deg, 1, 254, seed))


def test_rgg3d_shape():
    n = 1 << 18
    u, v, w = graphgen.rgg3d(n, graphgen.rgg3d_radius(n, 16), 1, 254, seed=7)
    assert (u < v).all() and w.min() >= 1 and w.max() <= 254
    assert 14.0 < 2 * len(u) / n < 16.5        # boundary effects lower the degree a little
    # lexicographic (u, v) order and no duplicates
    key = u.astype(np.int64) * n + v
    assert (np.diff(key) > 0).all()
    # locality: ids are cell-major, so endpoints are close in id
    assert np.median(np.abs(v.astype(np.int64) - u)) < n / 100


def test_rhg_shape():
    n = 1 << 18
    u, v, w = graphgen.rhg(n, 16.0, 1, 254, seed=8)
    assert (u < v).all() and w.min() >= 1 and w.max() <= 254
    assert 14.0 < 2 * len(u) / n < 18.0
    key = u.astype(np.int64) * n + v
    assert (np.diff(key) > 0).all()
    deg = np.bincount(u, minlength=n) + np.bincount(v, minlength=n)
    # power law with exponent 3: a heavy tail (max degree far above the mean;
    # P(deg >= k) ~ k^-2, so about 1 % of the vertices have degree >= 10x mean / ~3)
    assert deg.max() > 100 * deg.mean()
    frac = (deg >= 8 * deg.mean()).mean()
    assert 1e-4 < frac < 5e-2
    # angular ids: most edges join vertices close in id
    assert np.median(np.abs(v.astype(np.int64) - u)) < n / 100


def test_determinism_and_seed_dependence():
    a = graphgen.rmat(14, 100000, seed=3)
    assert same(a, graphgen.rmat(14, 100000, seed=3))
    assert not same(a, graphgen.rmat(14, 100000, seed=4))


def test_gnm_shape():
    n, m = 1 << 12, 1 << 18
    u, v, w = graphgen.gnm(n, m, 1, 2**31 - 1, seed=1)
    assert (u != v).all() and u.min() >= 0 and u.max() < n and v.max() < n
    deg = np.bincount(u, minlength=n) + np.bincount(v, minlength=n)
    assert abs(deg.mean() - 2 * m / n) < 1e-9
    assert deg.std() < 2 * np.sqrt(2 * m / n)          # Poisson-like
    assert w.min() >= 1 and w.max() <= 2**31 - 1


def test_rmat_shape():
    scale, m = 16, 1 << 20
    u, v, w = graphgen.rmat(scale, m, permute=False, seed=2)
    # top bit of (u, v) is the first quadrant choice: P(0,0)=a, P(0,1)=b, ...
    q = (u.astype(np.int64) >> (scale - 1)) * 2 + (v.astype(np.int64) >> (scale - 1))
    freq = np.bincount(q, minlength=4) / m
    assert np.allclose(freq, [0.57, 0.19, 0.19, 0.05], atol=0.003)
    assert w.min() == 1 and w.max() == 255
    # the Feistel map is a bijection on [0, 2^scale)
    for s in (10, 11):
        p = graphgen.rmat_permute(s, 2, np.arange(1 << s))
        assert (np.sort(p) == np.arange(1 << s)).all()


def test_grid_shape():
    u, v, w = graphgen.grid(200, 300, 0.8, 0, 10**6, 10**6, seed=3)
    cand = 200 * 299 + 199 * 300
    assert abs(len(u) / cand - 0.8) < 0.01
    d = v - u
    assert set(np.unique(d)) <= {1, 300}
    assert (w == 10**6).all()


def test_rgg_shape():
    n = 1 << 15
    r = graphgen.rgg_radius(n, 8.0)
    u, v, w = graphgen.rgg2d(n, r, 1e6, seed=4)
    assert (u < v).all()
    assert 7.0 < 2 * len(u) / n < 8.2                    # boundary effects lower it a bit
    assert w.max() <= int(np.ceil(1e6 * r))
    key = u.astype(np.int64) * n + v
    assert (np.diff(key) > 0).all()                     # lexicographic (i, j)


def test_star_forest_shape():
    u, v, w, n = graphgen.star_forest(50, 3, 2, 7, seed=5)
    assert n == 50 * 4 + 7 and len(u) == len(v) == len(w) == 50 * 3 * 2
    assert (u != v).all() and u.min() >= 0 and max(u.max(), v.max()) < n
    assert (w >= 1).all() and (w < 1000).all()
    # every vertex of an edge has degree 2 (leaf) or 6 (hub), and there are 50 hubs
    deg = np.bincount(np.concatenate([u, v]), minlength=n)
    assert sorted(set(deg.tolist())) == [0, 2, 6] and (deg == 6).sum() == 50
