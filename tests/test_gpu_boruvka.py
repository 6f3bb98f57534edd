"""Parity of the HIP Borůvka path against the CPU oracle (needs a GPU).

Bar: the MSF mask must equal the oracle's byte for byte and the 64-bit total
must be equal (integer work: bit-exact).  Per-round live-vertex and found-edge
counts must equal the plain round oracle (oracle.boruvka_rounds)."""
import hashlib

import numpy as np
import pytest

import graphgen
import oracle
from gpu_util import banner, golden_hashes, gpu_msf, sha

pytestmark = pytest.mark.gpu


def check_against_oracle(u, v, w, n, rounds=False, **kw):
    mask, total, stats = gpu_msf(u, v, w, n, **kw)
    rm, rt, rc = oracle.kruskal(u, v, w, n)
    assert (mask == rm).all(), f"mask differs at {np.nonzero(mask != rm)[0][:10]}"
    assert total == rt and stats["msf_edges"] == rc
    if rounds:
        _, _, orr = oracle.boruvka_rounds(u, v, w, n)
        assert stats["round_live"] == [r["live"] for r in orr]
        assert stats["round_found"] == [r["found"] for r in orr]
    return stats


def test_golden_hand_example(golden):
    g = golden("hand_example_7v.txt")
    banner("hand example")
    mask, total, stats = gpu_msf(g["u"], g["v"], g["w"], g["n"])
    assert (mask == g["mask"]).all() and total == g["total"]
    assert stats["msf_edges"] == g["count"]
    assert stats["round_live"] == [r["live"] for r in g["rounds"]]
    assert stats["round_found"] == [r["found"] for r in g["rounds"]]


@pytest.mark.parametrize("wmax", [0, 3, 255, 2**32 - 1])
def test_tiny_random_vs_brute_force(wmax):
    banner(f"tiny random wmax={wmax}")
    rng = np.random.default_rng(1000 + (wmax % 1000))
    for _ in range(60):
        n = int(rng.integers(1, 9))
        m = int(rng.integers(0, 14))
        u = rng.integers(0, n, m).astype(np.int32)
        v = rng.integers(0, n, m).astype(np.int32)
        w = rng.integers(0, wmax + 1, m, dtype=np.uint64).astype(np.uint32)
        mask, total, _ = gpu_msf(u, v, w, n)
        bm, bt = oracle.brute_force(u, v, w, n)
        assert (mask == bm).all() and total == bt, (u, v, w)


def test_closed_forms():
    banner("closed forms")
    k = 1000
    u = np.arange(k, dtype=np.int32)
    v = ((u + 1) % k).astype(np.int32)
    mask, total, _ = gpu_msf(u, v, np.full(k, 9, np.uint32), k)     # cycle, equal weights
    assert mask[:-1].all() and mask[-1] == 0 and total == 9 * (k - 1)
    # a path of 2^20 equal-weight edges, listed in order: every vertex but 0 picks
    # its lower edge, so round 0 leaves one chain 2^20 deep for pointer jumping
    k = 1 << 20
    u = np.arange(k - 1, dtype=np.int32)
    mask, total, st = gpu_msf(u, u + 1, np.full(k - 1, 3, np.uint32), k)
    assert mask.all() and total == 3 * (k - 1) and st["rounds"] >= 1
    n = 60                                                           # K_n, equal weights
    pairs = [(i, j) for i in range(n) for j in range(i + 1, n)]
    u = np.array([p[0] for p in pairs], np.int32)
    v = np.array([p[1] for p in pairs], np.int32)
    mask, total, _ = gpu_msf(u, v, np.full(len(pairs), 7, np.uint32), n)
    assert (mask == (u == 0)).all() and total == 7 * (n - 1)
    mask, total, st = gpu_msf(np.arange(50, dtype=np.int32), np.arange(50, dtype=np.int32),
                              np.ones(50, np.uint32), 50)            # only self-loops
    assert not mask.any() and total == 0 and st["msf_edges"] == 0
    mask, total, _ = gpu_msf(np.zeros(99, np.int32), np.arange(1, 100, dtype=np.int32),
                             np.arange(99, dtype=np.uint32)[::-1].copy(), 100)  # star
    assert mask.all() and total == sum(range(99))
    mask, total, st = gpu_msf(np.zeros(0, np.int32), np.zeros(0, np.int32),
                              np.zeros(0, np.uint32), 10)            # no edges
    assert total == 0 and st["msf_edges"] == 0


@pytest.mark.parametrize("kind,size", [("gnm", 12), ("gnm", 17), ("rmat", 14), ("rmat", 18),
                                       ("grid", 0), ("grid255", 0), ("rgg", 0), ("rgg3d", 17),
                                       ("rhg", 17), ("rhg", 12)])
def test_midsize_families_with_rounds(kind, size):
    banner(f"midsize {kind} {size}")
    if kind == "gnm":
        n = 1 << size
        u, v, w = graphgen.gnm(n, 8 * n + 1237, 1, 2**31 - 1, seed=size)
    elif kind == "rmat":
        n = 1 << size
        u, v, w = graphgen.rmat(size, 16 * n - 77, wlo=1, whi=255, seed=size)
    elif kind.startswith("grid"):
        n = 301 * 277
        u, v, w = graphgen.grid(301, 277, 0.8, 1 if kind == "grid255" else 0,
                                1 if kind == "grid255" else 10**6,
                                255 if kind == "grid255" else 10**6, seed=3)
    elif kind == "rgg3d":
        n = (1 << size) + 5
        u, v, w = graphgen.rgg3d(n, graphgen.rgg3d_radius(n, 16), 1, 254, seed=size)
    elif kind == "rhg":
        n = (1 << size) + 3
        u, v, w = graphgen.rhg(n, 16.0, 1, 254, seed=size)
    else:
        n = 90001
        u, v, w = graphgen.rgg2d(n, graphgen.rgg_radius(n, 8), 1e6, seed=4)
    check_against_oracle(u, v, w, n, rounds=True)


@pytest.mark.parametrize("order", ["sorted", "shuffled", "reversed", "swapped", "long_range",
                                   "ragged", "small_n", "loops_and_copies"])
def test_local_graph_edge_orders(order):
    """Graphs that pass the locality sample take round 0's lightest edges in a
    sliding LDS window over the ids; edges in any order, or far outside the
    window, must give the same forest (only the speed depends on the order)."""
    banner(f"locality window, edge order {order}")
    rng = np.random.default_rng(41)
    # the window kernels take graphs with a tile (8192 edges) for every
    # resident workgroup, i.e. at least 2^21 edges on this chip
    if order == "small_n":      # fewer vertices than a window: a local multigraph
        n = 6000
        m = (1 << 21) + 4099
        u = np.sort(rng.integers(0, n, m)).astype(np.int32)
        v = ((u.astype(np.int64) + rng.integers(1, 40, m)) % n).astype(np.int32)
        w = rng.integers(1, 256, m).astype(np.uint32)
    else:
        n = 600001
        u, v, w = graphgen.rgg2d(n, graphgen.rgg_radius(n, 8), 1e6, seed=4)
    if order == "shuffled":
        p = rng.permutation(len(u))
        u, v, w = u[p], v[p], w[p]
    elif order == "reversed":
        u, v, w = u[::-1].copy(), v[::-1].copy(), w[::-1].copy()
    elif order == "swapped":    # every other edge stored as (v, u)
        s = np.arange(len(u)) % 2 == 1
        u, v = np.where(s, v, u).astype(np.int32), np.where(s, u, v).astype(np.int32)
    elif order == "long_range":  # 2 % of the edges join random far-apart ids
        k = len(u) // 50
        at = np.sort(rng.choice(len(u), k, replace=False))
        u = u.copy()
        v = v.copy()
        v[at] = rng.integers(0, n, k).astype(np.int32)
    elif order == "loops_and_copies":   # 10 % self-loops and 10 % heavier parallel copies
        k = len(u) // 10
        at = np.sort(rng.choice(len(u), 2 * k, replace=False))
        u = u.copy()
        v = v.copy()
        w = w.copy()
        v[at[:k]] = u[at[:k]]                         # self-loops in place
        src = at[k:] - 1                              # a copy of the edge before, heavier
        u[at[k:]], v[at[k:]] = v[src], u[src]
        w[at[k:]] = np.minimum(w[src].astype(np.uint64) + 1, 2**32 - 1).astype(np.uint32)
    elif order == "ragged":     # not a multiple of the vector width or the tile
        u, v, w = u[:len(u) - 8192 - 3], v[:len(v) - 8192 - 3], w[:len(w) - 8192 - 3]
    assert len(u) >= 1 << 21
    check_against_oracle(u, v, w, n, rounds=True)


def test_out_of_range_id_in_a_local_graph():
    import paper_2302_12199_amd as msf
    banner("out of range id in a local graph")
    n = 600001
    u, v, w = graphgen.rgg2d(n, graphgen.rgg_radius(n, 8), 1e6, seed=4)
    for at, bad in ((len(u) // 2, n), (len(u) - 1, 2**31 - 1), (5, -1)):
        uu = u.copy()
        uu[at] = bad
        with pytest.raises(msf.MSFError) as e:
            gpu_msf(uu, v, w, n)
        assert e.value.status == msf.ERANGE


@pytest.mark.parametrize("tail", [0, 1, 2, 100, 1024])
@pytest.mark.parametrize("kind", ["gnm", "grid", "rmat_filter"])
def test_tail_threshold(kind, tail):
    """The single-workgroup tail runs the same rounds (Sec. II-C) on the
    lightest edge of each vertex pair, so where it takes over changes neither
    the forest nor the per-round trace; 1 never uses it."""
    banner(f"tail threshold {tail} on {kind}")
    if kind == "gnm":
        n = 1 << 14
        u, v, w = graphgen.gnm(n, 8 * n + 11, 1, 2**31 - 1, seed=14)
        check_against_oracle(u, v, w, n, rounds=True, tail_threshold=tail)
    elif kind == "grid":
        n = 301 * 277
        u, v, w = graphgen.grid(301, 277, 0.8, 1, 1, 255, seed=3)
        check_against_oracle(u, v, w, n, rounds=True, tail_threshold=tail)
    else:
        n = 1 << 16
        u, v, w = graphgen.rmat(16, 32 * n, wlo=1, whi=2**31 - 1, seed=16)
        check_against_oracle(u, v, w, n, algo="filter", min_split_edges=20000,
                             tail_threshold=tail)


def test_config_gnm_2p16_2p20():
    banner("GNM n=2^16 m=2^20 (oracle live)")
    u, v, w, n = graphgen.workload("gnm_n2^16_m2^20")
    check_against_oracle(u, v, w, n, rounds=True)


FULL = ["rmat_n2^24_m2^28_w255", "grid_4096x4096_keep0.8_w1e6", "grid_4096x4096_keep0.8_w255",
        "rgg2d_n2^24_deg8", "rmat_n2^22_m2^28_w2^31", "rgg3d_n2^24_deg16_w254",
        "rhg_n2^24_deg16_g3_w254"]


@pytest.mark.parametrize("name", FULL)
def test_fullsize_matches_stored_oracle(name):
    ref = golden_hashes()[name]
    banner(f"full size {name} (stored oracle hash)")
    u, v, w, n = graphgen.workload(name)
    assert len(u) == ref["m"] and n == ref["n"]
    assert hashlib.sha256(u.tobytes() + v.tobytes() + w.tobytes()).hexdigest() == \
        ref["input_sha256"], "the generator produced a different input on this machine"
    mask, total, stats = gpu_msf(u, v, w, n)
    assert total == ref["total"] and stats["msf_edges"] == ref["msf_edges"]
    assert sha(mask) == ref["mask_sha256"]
    # n_{r+1} <= n_r / 2 for live vertices (Sec. II-C)
    live = stats["round_live"]
    assert all(b <= a // 2 for a, b in zip(live, live[1:]))


def test_repeat_runs_bit_identical():
    banner("determinism")
    u, v, w = graphgen.rmat(18, 1 << 22, wlo=1, whi=15, seed=77)
    first = gpu_msf(u, v, w, 1 << 18)
    for _ in range(3):
        again = gpu_msf(u, v, w, 1 << 18)
        assert (again[0] == first[0]).all() and again[1] == first[1]


def test_metamorphic():
    banner("metamorphic")
    rng = np.random.default_rng(9)
    n = 20000
    u, v, w = graphgen.gnm(n, 150000, 1, 50, seed=9)
    mask, total, _ = gpu_msf(u, v, w, n)
    m2, _, _ = gpu_msf(u, v, (2 * w + 1).astype(np.uint32), n)
    assert (m2 == mask).all()
    p = rng.permutation(n).astype(np.int32)
    m2, t2, _ = gpu_msf(p[u], p[v], w, n)
    assert (m2 == mask).all() and t2 == total
    uu = np.concatenate([u, u[:5000], np.arange(300, dtype=np.int32)])
    vv = np.concatenate([v, v[:5000], np.arange(300, dtype=np.int32)])
    ww = np.concatenate([w, w[:5000], np.zeros(300, np.uint32)])
    m2, t2, _ = gpu_msf(uu, vv, ww, n)
    assert (m2[:len(u)] == mask).all() and not m2[len(u):].any() and t2 == total


def test_out_of_range_ids_reported():
    import paper_2302_12199_amd as msf
    banner("out of range")
    u = np.array([0, 1, 2], np.int32)
    v = np.array([1, 2, 3], np.int32)
    with pytest.raises(msf.MSFError) as e:
        gpu_msf(u, v, np.ones(3, np.uint32), 3)
    assert e.value.status == msf.ERANGE
    with pytest.raises(msf.MSFError) as e:
        gpu_msf(np.array([0, -5], np.int32), np.array([1, 1], np.int32), np.ones(2, np.uint32), 3)
    assert e.value.status == msf.ERANGE


def test_library_allocated_workspace_and_sparse_large_n():
    import torch
    import paper_2302_12199_amd as msf
    from gpu_util import to_dev
    banner("library workspace, large sparse n")
    n = 1 << 26
    rng = np.random.default_rng(4)
    u = rng.integers(0, n, 5000).astype(np.int32)
    v = rng.integers(0, n, 5000).astype(np.int32)
    w = rng.integers(0, 3, 5000).astype(np.uint32)
    tu, tv, tw = to_dev(u, v, w)
    mask = torch.empty(5000, dtype=torch.uint8, device="cuda:0")
    torch.cuda.synchronize()
    rc, total = msf.compute_raw(tu.data_ptr(), tv.data_ptr(), tw.data_ptr(), 5000, n,
                                mask.data_ptr())   # workspace NULL: library allocates
    assert rc == msf.OK
    rm, rt, _ = oracle.kruskal(u, v, w, n)
    assert (mask.cpu().numpy() == rm).all() and total == rt


def test_single_vertex_and_two_vertex_multigraph():
    banner("n=1, n=2")
    mask, total, _ = gpu_msf(np.zeros(5, np.int32), np.zeros(5, np.int32),
                             np.arange(5, dtype=np.uint32), 1)
    assert not mask.any() and total == 0
    u = np.array([0, 1, 0, 1, 0], np.int32)
    v = np.array([1, 0, 1, 0, 0], np.int32)
    w = np.array([5, 3, 3, 9, 0], np.uint32)
    mask, total, _ = gpu_msf(u, v, w, 2)
    assert list(mask) == [0, 1, 0, 0, 0] and total == 3


def test_compose_pass_after_compaction_keeps_all_positions():
    # regression: a relabel pass that only composes maps on an already
    # compacted layout must keep every position (grids reach this path)
    banner("compose after compaction")
    for rows, cols in [(64, 64), (301, 277)]:
        u, v, w = graphgen.grid(rows, cols, 0.8, 1, 1, 255, seed=3)
        check_against_oracle(u, v, w, rows * cols, rounds=True)


def test_pass_leaving_no_live_edge_ends_the_rounds():
    # more components than the tail takes, and none of them joined by an edge:
    # the relabel pass leaves no live edge, which the next round's counters show
    banner("5000 disjoint stars (one round, no tail)")
    u, v, w, n = graphgen.star_forest(5000, 3, 3, 777, seed=90)
    st = check_against_oracle(u, v, w, n, rounds=True)
    assert len(st["round_live"]) == 1
