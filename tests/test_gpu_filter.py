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


def check_filter(u, v, w, n, seed=1, sample=4096, q=0.5, min_split=2000, sparse_degree=4,
                 pivot="quantile"):
    mask, total, st = gpu_msf(u, v, w, n, algo="filter", pivot=pivot, quantile=q, seed=seed,
                              sample_size=sample, min_split_edges=min_split,
                              sparse_degree=sparse_degree)
    km, kt, kc = oracle.kruskal(u, v, w, n)
    assert (mask == km).all(), f"mask differs at {np.nonzero(mask != km)[0][:10]}"
    assert total == kt and st["msf_edges"] == kc
    _, _, trace = oracle.filter_boruvka(u, v, w, n, seed=seed, sample=sample, q=q,
                                        min_split=min_split, sparse_degree=sparse_degree)
    got = [{k: s[k] for k in ("edges", "pivot", "light", "kept")} for s in st["splits"]]
    assert got == trace[:len(got)] and len(got) == min(len(trace), 64)
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
