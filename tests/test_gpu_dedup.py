"""Parallel-edge removal in the Borůvka rounds (needs a GPU).

Every policy must give the oracle's MSF bit for bit and the oracle's
per-round live-vertex and found-edge counts (removing a heavier parallel
edge never changes a lightest incident edge).  With exact removal every
compacted round must see exactly the oracle's number of distinct vertex
pairs; the per-tile prefilter must land between that and the count with all
parallel edges kept."""
import numpy as np
import pytest

import graphgen
import oracle
from gpu_util import banner, gpu_msf

pytestmark = pytest.mark.gpu

POLICIES = ["never", "local", "exact", "auto"]


def family(kind):
    if kind == "gnm":
        n = 1 << 15
        return (*graphgen.gnm(n, 12 * n + 5, 1, 2**31 - 1, seed=3), n)
    if kind == "rmat":
        n = 1 << 16
        return (*graphgen.rmat(16, 24 * n - 3, wlo=1, whi=255, seed=4), n)
    if kind == "grid255":
        return (*graphgen.grid(333, 301, 0.8, 1, 1, 255, seed=5), 333 * 301)
    if kind == "rgg":
        n = 150001
        return (*graphgen.rgg2d(n, graphgen.rgg_radius(n, 8), 1e6, seed=6), n)
    if kind == "rgg3d":
        n = 1 << 17
        return (*graphgen.rgg3d(n, graphgen.rgg3d_radius(n, 16), 1, 254, seed=7), n)
    n = (1 << 17) + 1
    return (*graphgen.rhg(n, 16.0, 1, 254, seed=8), n)


@pytest.mark.parametrize("kind", ["gnm", "rmat", "grid255", "rgg", "rgg3d", "rhg"])
def test_policies_parity_and_edge_counts(kind):
    u, v, w, n = family(kind)
    rm, rt, rc = oracle.kruskal(u, v, w, n)
    _, _, orr = oracle.boruvka_rounds(u, v, w, n)
    counts = {}
    for pol in POLICIES:
        banner(f"dedup {kind} policy={pol}")
        mask, total, st = gpu_msf(u, v, w, n, dedup=pol)
        assert (mask == rm).all(), (pol, np.nonzero(mask != rm)[0][:10])
        assert total == rt and st["msf_edges"] == rc
        assert st["round_live"] == [r["live"] for r in orr], pol
        assert st["round_found"] == [r["found"] for r in orr], pol
        counts[pol] = st
    # rounds run by the main loop (more than 1024 labels) after round 0
    main = [r for r in range(1, len(orr)) if orr[r]["vertices"] > 1024]
    for r in main:
        assert counts["never"]["round_edges"][r] == orr[r]["edges"]
        assert counts["exact"]["round_edges"][r] == orr[r]["pairs"], (kind, r)
        assert orr[r]["pairs"] <= counts["local"]["round_edges"][r] <= orr[r]["edges"]


@pytest.mark.parametrize("pol", POLICIES)
def test_appended_parallel_copies_never_enter_the_msf(pol):
    banner(f"dedup metamorphic policy={pol}")
    n = 40000
    u, v, w = graphgen.rgg2d(n, graphgen.rgg_radius(n, 8), 1e6, seed=11)
    mask, total, _ = gpu_msf(u, v, w, n, dedup=pol)
    rm, rt, _ = oracle.kruskal(u, v, w, n)
    assert (mask == rm).all() and total == rt
    # copies with equal or larger weight and a larger id, reversed or not
    k = len(u)
    rng = np.random.default_rng(2)
    sel = rng.integers(0, k, 3 * k)
    flip = rng.random(3 * k) < 0.5
    uu = np.concatenate([u, np.where(flip, v[sel], u[sel])]).astype(np.int32)
    vv = np.concatenate([v, np.where(flip, u[sel], v[sel])]).astype(np.int32)
    ww = np.concatenate([w, w[sel] + rng.integers(0, 3, 3 * k).astype(np.uint32)])
    m2, t2, _ = gpu_msf(uu, vv, ww, n, dedup=pol)
    assert (m2[:k] == mask).all() and not m2[k:].any() and t2 == total


def test_exact_policy_fullsize_rgg_matches_stored_oracle():
    from gpu_util import golden_hashes, sha
    name = "rgg2d_n2^24_deg8"
    ref = golden_hashes()[name]
    banner(f"dedup exact full size {name}")
    u, v, w, n = graphgen.workload(name)
    mask, total, st = gpu_msf(u, v, w, n, dedup="exact")
    assert total == ref["total"] and st["msf_edges"] == ref["msf_edges"]
    assert sha(mask) == ref["mask_sha256"]
