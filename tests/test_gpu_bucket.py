"""Parity of the bucketed round 0 against the CPU oracle (needs a GPU).

Round 0 on the caller's arrays runs either directly on the edge list
(round0="edges") or by vertex buckets (round0="buckets", where the graph
qualifies: 2^21 <= n <= 2^24, 2^22 <= m < 2^31; round0="auto" picks buckets
there unless most sampled edges join nearby ids).  Both must give the
oracle's mask byte for byte and its 64-bit total, and the same per-round
counts (the rounds are the same Borůvka rounds; only their data layout
differs)."""
import numpy as np
import pytest

import graphgen
import oracle
from gpu_util import banner, gpu_msf

pytestmark = pytest.mark.gpu


def run(u, v, w, n, round0, **kw):
    import paper_2302_12199_amd as msf
    msf.profile_enable(True)
    msf.profile_reset()
    try:
        mask, total, stats = gpu_msf(u, v, w, n, round0=round0, **kw)
        prof = msf.profile_read()
    finally:
        msf.profile_enable(False)
    return mask, total, stats, prof.get("bucket_min", {}).get("launches", 0)


def both(u, v, w, n, expect_buckets=True, **kw):
    rm, rt, rc = oracle.kruskal(u, v, w, n)
    mb, tb, sb, lb = run(u, v, w, n, "buckets", **kw)
    me, te, se, le = run(u, v, w, n, "edges", **kw)
    assert (lb > 0) == expect_buckets and le == 0
    assert (mb == rm).all(), f"bucketed mask differs at {np.nonzero(mb != rm)[0][:10]}"
    assert (me == rm).all(), f"edge-list mask differs at {np.nonzero(me != rm)[0][:10]}"
    assert tb == rt and te == rt and sb["msf_edges"] == rc and se["msf_edges"] == rc
    assert sb["round_live"] == se["round_live"] and sb["round_found"] == se["round_found"]
    return sb


@pytest.mark.parametrize("n,m,whi,seed", [(1 << 21, 1 << 22, 2**31 - 1, 11),
                                          (1 << 21, 1 << 23, 3, 12),
                                          (1 << 22, 1 << 23, 255, 13)])
def test_gnm(n, m, whi, seed):
    banner(f"bucketed round 0, gnm n={n} m={m} w<= {whi}")
    u, v, w = graphgen.gnm(n, m, 1, whi, seed=seed)
    both(u, v, w, n)


@pytest.mark.parametrize("scale,m,whi", [(21, 1 << 23, 255), (22, 1 << 22, 2**31 - 1)])
def test_rmat_hubs(scale, m, whi):
    banner(f"bucketed round 0, rmat scale {scale} m={m}")
    u, v, w = graphgen.rmat(scale, m, wlo=1, whi=whi, seed=21)
    both(u, v, w, 1 << scale)


def test_ragged_sizes_self_loops_and_parallel_edges():
    # n not a multiple of the bucket width, m not a multiple of the tile or of 4
    banner("bucketed round 0, ragged sizes, self-loops, parallel edges")
    n = (1 << 21) + 12345
    m = (1 << 22) + 4093
    rng = np.random.default_rng(5)
    u = rng.integers(0, n, m).astype(np.int32)
    v = rng.integers(0, n, m).astype(np.int32)
    loops = rng.random(m) < 0.05
    v[loops] = u[loops]
    dup = np.nonzero(rng.random(m) < 0.05)[0]
    src = rng.integers(0, m, len(dup))
    u[dup], v[dup] = v[src], u[src]                 # reversed copies of other edges
    w = rng.integers(0, 1000, m).astype(np.uint32)
    u[-1], v[-1] = n - 1, 0                          # the last vertex and the last tile
    both(u, v, w, n)


def test_stars_reach_the_tail_after_round_zero():
    # 500 hub stars of weight-1 edges joined by heavier leaf-to-leaf edges:
    # round 0 leaves exactly the 500 stars, which go to the single-workgroup tail
    banner("bucketed round 0, 500 stars (one round, then the tail)")
    n = 1 << 21
    hubs = 500
    leaves = np.arange(hubs, n, dtype=np.int32)
    rng = np.random.default_rng(6)
    extra = (1 << 22) - len(leaves)
    u = np.concatenate([leaves % hubs, rng.integers(hubs, n, extra)]).astype(np.int32)
    v = np.concatenate([leaves, rng.integers(hubs, n, extra)]).astype(np.int32)
    w = np.concatenate([np.ones(len(leaves), np.uint32),
                        rng.integers(2, 1000, extra).astype(np.uint32)])
    perm = rng.permutation(len(u))
    st = both(u[perm], v[perm], w[perm], n)
    assert st["round_live"][1] == hubs


def test_out_of_range_ids_reported():
    import paper_2302_12199_amd as msf
    banner("bucketed round 0, out-of-range ids")
    n = 1 << 21
    u, v, w = graphgen.gnm(n, 1 << 22, 1, 100, seed=7)
    for pos, bad in [(len(u) - 1, n), (12345, -3)]:
        uu = u.copy()
        uu[pos] = bad
        with pytest.raises(msf.MSFError) as e:
            gpu_msf(uu, v, w, n, round0="buckets")
        assert e.value.status == msf.ERANGE


def test_filter_base_case_on_the_callers_arrays():
    # a sparse graph (2m/n <= 4) goes to the base case unsplit, on the caller's arrays
    banner("bucketed round 0 inside Filter-Borůvka")
    n = 1 << 21
    u, v, w = graphgen.gnm(n, 1 << 22, 1, 2**31 - 1, seed=8)
    rm, rt, _ = oracle.kruskal(u, v, w, n)
    mask, total, _, launches = run(u, v, w, n, "buckets", algo="filter")
    assert launches > 0
    assert (mask == rm).all() and total == rt


def test_workspace_sizes():
    import paper_2302_12199_amd as msf
    banner("bucketed round 0, workspace sizes")
    m, n = 1 << 22, 1 << 21
    assert msf.workspace_bytes(m, n) == msf.workspace_bytes(m, n, round0="buckets")
    assert msf.workspace_bytes(m, n) - msf.workspace_bytes(m, n, round0="edges") >= 24 * m
    assert msf.workspace_bytes(1 << 20, 1 << 16) == msf.workspace_bytes(1 << 20, 1 << 16,
                                                                       round0="edges")
    # too small for buckets: the edge-list round 0 runs even when buckets are asked for
    u, v, w = graphgen.gnm(1 << 16, 1 << 20, 1, 2**31 - 1, seed=9)
    both(u, v, w, 1 << 16, expect_buckets=False)


def test_auto_choice_follows_id_locality():
    banner("round0=auto: random ids -> buckets, grid ids -> edge list")
    n = 1 << 21
    u, v, w = graphgen.gnm(n, 1 << 22, 1, 2**31 - 1, seed=10)
    rm, rt, _ = oracle.kruskal(u, v, w, n)
    mask, total, _, launches = run(u, v, w, n, "auto")
    assert launches > 0 and (mask == rm).all() and total == rt
    rows = cols = 2048
    u, v, w = graphgen.grid(rows, cols, 0.8, 1, 1, 255, seed=11)
    assert len(u) >= 1 << 22
    rm, rt, _ = oracle.kruskal(u, v, w, rows * cols)
    mask, total, _, launches = run(u, v, w, rows * cols, "auto")
    assert launches == 0 and (mask == rm).all() and total == rt
    both(u, v, w, rows * cols)


def test_pass_leaving_no_live_edge_ends_the_rounds():
    # 2^19 disjoint 4-vertex stars, each edge three times: the bucketed round 0
    # merges every star and its pass leaves no live edge
    banner("bucketed round 0, 2^19 disjoint stars (one round)")
    u, v, w, n = graphgen.star_forest(1 << 19, 3, 3, 12345, seed=91)
    assert n >= 1 << 21 and len(u) >= 1 << 22
    st = both(u, v, w, n)
    assert len(st["round_live"]) == 1
