"""Parity of the HIP Filter-Borůvka path (needs a GPU).

Final result: the MSF mask byte for byte and the total, against Kruskal.
Every split: the pivot key, the light-edge count and the number of heavy
edges surviving the filter, against the step-by-step CPU reference
(oracle.filter_boruvka), which draws the same pivot samples from its own
SplitMix64 implementation."""
import numpy as np
import pytest

import graphgen
import oracle
from gpu_util import banner, golden_hashes, gpu_msf, sha

pytestmark = pytest.mark.gpu


def assert_features_close(got, ref, sample):
    """The sampler's 16 pivot-network features (single precision on the
    device) against the float64 oracle.  Bounds, from the arithmetic:
    statistics of L(w) = log2(1 + w) / 32 come from one single-precision
    log2 (about one ulp of a result below 1) of a rounded conversion, so
    |error| <= 1e-6; the mean is a single-precision sum of up to 8192 such
    terms (per-thread sums, then a tree), |error| <= 2e-6; the deviation is
    sqrt(E[L^2] - mean^2) with both moments in single precision, so its
    square is compared, |error| <= 1e-5; the tie and repeat fractions are
    exact integer counts, compared as counts."""
    g, r = np.asarray(got, np.float64), np.asarray(ref, np.float64)
    idx = [0, 1, 2, 3, 4, 8, 9, 10, 11, 12, 13]
    np.testing.assert_allclose(g[idx], r[idx], rtol=0, atol=1e-6)
    assert abs(g[5] - r[5]) <= 2e-6, (g[5], r[5])
    assert abs(g[6] ** 2 - r[6] ** 2) <= 1e-5, (g[6], r[6])
    pairs = max(sample - 1, 1)
    assert round(g[7] * pairs) == round(r[7] * pairs)
    ends = 2 * min(sample, 2048) - 1
    assert round(g[14] * ends) == round(r[14] * ends)
    assert g[15] == 1.0


def check_filter(u, v, w, n, seed=1, sample=4096, q=0.5, min_split=2000, sparse_degree=4,
                 pivot="quantile", definition=False):
    mask, total, st = gpu_msf(u, v, w, n, algo="filter", pivot=pivot, quantile=q, seed=seed,
                              sample_size=sample, min_split_edges=min_split,
                              sparse_degree=sparse_degree)
    km, kt, kc = oracle.kruskal(u, v, w, n)
    assert (mask == km).all(), f"mask differs at {np.nonzero(mask != km)[0][:10]}"
    assert total == kt and st["msf_edges"] == kc
    _, _, trace = oracle.filter_boruvka(u, v, w, n, seed=seed, sample=sample, q=q,
                                        min_split=min_split, sparse_degree=sparse_degree)
    if definition:      # the second, union-find-free formulation of the trace
        from oracle.filter_def import trace_by_definition
        td = trace_by_definition(u, v, w, n, seed=seed, sample=sample, q=q,
                                 min_split=min_split, sparse_degree=sparse_degree)
        assert [{k: t[k] for k in ("edges", "pivot", "light", "kept")} for t in td] == \
            [{k: t[k] for k in ("edges", "pivot", "light", "kept")} for t in trace]
    got = [{k: s[k] for k in ("edges", "pivot", "light", "kept")} for s in st["splits"]]
    want = [{k: t[k] for k in ("edges", "pivot", "light", "kept")} for t in trace]
    assert got == want[:len(got)] and len(got) == min(len(trace), 64)
    for s, t in zip(st["splits"], trace):
        assert_features_close(s["features"], t["features"], sample)
    if st["splits"]:
        assert st["top_features"] == st["splits"][0]["features"]
    return st


@pytest.mark.parametrize("kind", ["rmat", "gnm", "grid"])
def test_filter_midsize_with_trace(kind):
    banner(f"filter midsize {kind}")
    if kind == "rmat":
        n = 1 << 14
        u, v, w = graphgen.rmat(14, 64 * n + 11, wlo=1, whi=2**31 - 1, seed=31)
    elif kind == "gnm":
        n = 20000
        u, v, w = graphgen.gnm(n, 400001, 1, 1000, seed=32)
    else:
        n = 200 * 150
        u, v, w = graphgen.grid(200, 150, 0.8, 1, 1, 255, seed=33)
    st = check_filter(u, v, w, n)
    assert st["levels"] >= 1 or kind == "grid"


@pytest.mark.parametrize("q", [0.0, 1e-6, 0.01, 0.5, 0.99, 1.0])
def test_filter_any_quantile_same_msf(q):
    banner(f"filter quantile {q}")
    n = 1 << 13
    u, v, w = graphgen.rmat(13, 40 * n, wlo=1, whi=255, seed=40)
    check_filter(u, v, w, n, q=q, min_split=5000)


@pytest.mark.parametrize("sample", [1, 3, 100, 8192])
def test_filter_sample_sizes(sample):
    banner(f"filter sample {sample}")
    n = 5000
    u, v, w = graphgen.gnm(n, 120000, 1, 2**31 - 1, seed=sample)
    check_filter(u, v, w, n, sample=sample, seed=sample + 7, min_split=3000)


@pytest.mark.parametrize("kind", ["gnm", "rmat"])
@pytest.mark.parametrize("sample", [1, 100, 4096, 8192])
def test_filter_features_match_oracle(kind, sample):
    """Every split's pivot-network features -- the top split reads the
    caller's arrays, deeper ones the compacted buffers in label space --
    against the float64 feature oracle on the same draws."""
    banner(f"filter features {kind} sample={sample}")
    if kind == "gnm":
        n = 6000
        u, v, w = graphgen.gnm(n, 150000, 1, 2**31 - 1, seed=50 + sample % 97)
    else:
        n = 1 << 13
        u, v, w = graphgen.rmat(13, 200000, wlo=1, whi=255, seed=60 + sample % 89)
    st = check_filter(u, v, w, n, sample=sample, seed=sample + 3, q=0.3, min_split=3000,
                      definition=True)
    assert len(st["splits"]) >= 2 and any(f["features"][13] > 0 for f in st["splits"])


@pytest.mark.parametrize("graph", ["gnm", "rmat"])
@pytest.mark.parametrize("retries,defer,sample,q", [(6, 0, 1, 0.5), (6, 0, 1, 0.2),
                                                    (0, 3000, 256, 0.3), (4, 3000, 16, 0.5),
                                                    (0, 10**6, 512, 0.5)])
def test_filter_variants_match_the_oracle(graph, retries, defer, sample, q):
    """The balanced-split retry and the deferral of small filtered sets: the
    MSF, every split (including its draws and handed-back edges), the
    features, and the counts of redraws, deferrals and base cases."""
    banner(f"filter variants {graph} retries={retries} defer={defer} sample={sample} q={q}")
    if graph == "gnm":
        n = 3000
        u, v, w = graphgen.gnm(n, 90000, 1, 2**31 - 1, seed=12)
    else:
        n = 1 << 13
        u, v, w = graphgen.rmat(13, 150000, wlo=1, whi=2**31 - 1, seed=13)
    mask, total, st = gpu_msf(u, v, w, n, algo="filter", pivot="quantile", quantile=q, seed=2,
                              sample_size=sample, min_split_edges=1000, split_retries=retries,
                              defer_edges=defer)
    km, kt, kc = oracle.kruskal(u, v, w, n)
    assert (mask == km).all() and total == kt and st["msf_edges"] == kc
    info = {}
    _, _, trace = oracle.filter_boruvka(u, v, w, n, seed=2, sample=sample, q=q, min_split=1000,
                                        retries=retries, defer=defer, info=info)
    keys = ("edges", "pivot", "light", "kept", "attempts", "deferred_in")
    assert [{k: s_[k] for k in keys} for s_ in st["splits"]] == \
        [{k: t[k] for k in keys} for t in trace[:64]]
    for s_, t in zip(st["splits"], trace):
        assert_features_close(s_["features"], t["features"], sample)
    assert st["pivot_retries"] == info["retries"] and st["deferrals"] == info["deferrals"]
    assert st["base_cases"] == info["base_cases"]


def test_filter_ties_and_selfloops():
    banner("filter ties")
    rng = np.random.default_rng(5)
    n = 3000
    u = rng.integers(0, n, 90000).astype(np.int32)
    v = rng.integers(0, n, 90000).astype(np.int32)
    w = rng.integers(0, 3, 90000).astype(np.uint32)      # massive ties, some self-loops
    check_filter(u, v, w, n, min_split=2000)


def test_filter_median_pivot_default_options():
    banner("filter median, defaults")
    n = 1 << 16
    u, v, w = graphgen.rmat(16, 1 << 21, wlo=1, whi=2**31 - 1, seed=41)
    mask, total, st = gpu_msf(u, v, w, n, algo="filter")
    km, kt, _ = oracle.kruskal(u, v, w, n)
    assert (mask == km).all() and total == kt


def test_filter_fullsize_rmat22_matches_stored_oracle():
    name = "rmat_n2^22_m2^28_w2^31"
    ref = golden_hashes()[name]
    banner(f"filter full size {name}")
    u, v, w, n = graphgen.workload(name)
    mask, total, st = gpu_msf(u, v, w, n, algo="filter")
    assert total == ref["total"] and st["msf_edges"] == ref["msf_edges"]
    assert sha(mask) == ref["mask_sha256"]
    assert st["levels"] >= 3


@pytest.mark.parametrize("name,pivot", [("rmat_n2^24_m2^28_w255", "median"),
                                        ("rmat_n2^24_m2^28_w255", "mlp"),
                                        ("rmat_n2^22_m2^28_w2^31", "mlp"),
                                        ("grid_4096x4096_keep0.8_w255", "median"),
                                        ("rgg2d_n2^24_deg8", "median")])
def test_filter_fullsize_other_workloads(name, pivot):
    """Full-size configurations through Filter-Borůvka (the shipped network or
    the median pivot) against the stored oracle masks."""
    import paper_2302_12199_amd as msf
    ref = golden_hashes()[name]
    banner(f"filter full size {name} pivot={pivot}")
    u, v, w, n = graphgen.workload(name)
    if pivot == "mlp":
        msf.load_pivot_model()
    try:
        mask, total, st = gpu_msf(u, v, w, n, algo="filter", pivot=pivot,
                                  min_split_edges=1 << 16)
    finally:
        msf.clear_pivot_model()
    assert total == ref["total"] and st["msf_edges"] == ref["msf_edges"]
    assert sha(mask) == ref["mask_sha256"]


def test_filter_out_of_range():
    import paper_2302_12199_amd as msf
    banner("filter out of range")
    n = 1000
    u, v, w = graphgen.gnm(n, 50000, 1, 100, seed=3)
    v = v.copy()
    v[12345] = n + 5
    with pytest.raises(msf.MSFError) as e:
        gpu_msf(u, v, w, n, algo="filter", min_split_edges=100)
    assert e.value.status == msf.ERANGE
