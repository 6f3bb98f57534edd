"""Parity of the batched persistent solver (needs a GPU): every graph's MSF
mask and total against the per-graph CPU oracle."""
import numpy as np
import pytest

import graphgen
import oracle
from gpu_util import banner, to_dev

pytestmark = pytest.mark.gpu


def oracle_batch(u, v, w, eo, vo):
    masks, totals = [], []
    for g in range(len(eo) - 1):
        a, b = eo[g], eo[g + 1]
        mk, t, _ = oracle.kruskal(u[a:b], v[a:b], w[a:b], int(vo[g + 1] - vo[g]))
        masks.append(mk)
        totals.append(t)
    return (np.concatenate(masks) if masks else np.zeros(0, np.uint8)), np.array(totals, np.uint64)


def make_batch(u, v, w, eo, vo, **kw):
    import paper_2302_12199_amd as msf
    tu, tv, tw = to_dev(u, v, w)
    return msf.Batch(tu, tv, tw, eo, vo, **kw)


def results(b):
    import torch
    torch.cuda.synchronize()
    m = int(b.eoff[-1].item()) if b.G else 0
    return b.mask[:m].cpu().numpy(), b.totals[:b.G].cpu().numpy().view(np.uint64)


@pytest.mark.parametrize("block,lds", [(1024, 0), (256, -1), (512, 1024), (1024, 4096),
                                       (512, 8000), (1024, 8000)])
def test_batch_matches_oracle(block, lds):
    import paper_2302_12199_amd as msf
    banner(f"batch block={block} lds={lds}")
    u, v, w, eo, vo = graphgen.batch_gnm(300, lo=8, hi=13, seed=11)
    rm, rt = oracle_batch(u, v, w, eo, vo)
    b = make_batch(u, v, w, eo, vo, options=msf.make_batch_options(block=block, lds_vertices=lds))
    b.launch()
    mask, totals = results(b)
    assert (totals == rt).all()
    assert (mask == rm).all()


@pytest.mark.parametrize("coop,workgroups", [(1 << 16, 0), (1 << 14, 0), (1 << 16, 24),
                                             (1 << 16, 3)])
def test_batch_cooperative_match_oracle(coop, workgroups):
    """Graphs with at least coop edges are solved by all workgroups of an XCD
    together, the rest by one workgroup each (LDS or a global slot); also with
    fewer workgroups than XCDs."""
    import paper_2302_12199_amd as msf
    banner(f"batch coop={coop} workgroups={workgroups}")
    u, v, w, eo, vo = graphgen.batch_gnm(160, lo=8, hi=15, dlo=2, dhi=40, seed=21)
    rm, rt = oracle_batch(u, v, w, eo, vo)
    b = make_batch(u, v, w, eo, vo,
                   options=msf.make_batch_options(block=512, lds_vertices=1024,
                                                  coop_edges=coop, workgroups=workgroups))
    for _ in range(2):                    # a second launch reuses the team blocks
        b.launch()
        mask, totals = results(b)
        assert (totals == rt).all()
        assert (mask == rm).all()


@pytest.mark.parametrize("hot_min,wave_min,coop", [(0, 0, 1 << 16), (4, 2, 1 << 15),
                                                   (-1, -1, 1 << 14), (1, 64, 1 << 14)])
def test_batch_tiers_match_oracle(hot_min, wave_min, coop):
    """The workgroup and XCD graph tiers with the vertex tiers of the
    lightest-edge search (block: LDS minima of a chunk's sampled frequent
    labels; wave: lanes sharing a label combined) at several thresholds,
    including every label in the block tier (hot_min 1) and a wave tier that
    never triggers (64)."""
    import paper_2302_12199_amd as msf
    wave_edges = -1
    banner(f"batch tiers hot_min={hot_min} wave_min={wave_min} coop={coop}")
    u, v, w, eo, vo = graphgen.batch_gnm(300, lo=8, hi=15, dlo=2, dhi=40, wlo=1, whi=40,
                                         seed=31)
    rm, rt = oracle_batch(u, v, w, eo, vo)
    opts = msf.make_batch_options(block=512, lds_vertices=4096, coop_edges=coop,
                                  wave_edges=wave_edges, hot_min=hot_min, wave_min=wave_min)
    b = make_batch(u, v, w, eo, vo, options=opts)
    for _ in range(2):
        b.launch()
        mask, totals = results(b)
        assert (totals == rt).all()
        assert (mask == rm).all()
    ticks = b.ticks.cpu().numpy().view(np.uint64)
    G = len(rt)
    assert (ticks[:G] >= ticks[G + 1:]).all()


@pytest.mark.skip(reason="the wave-per-graph tier hung the GPU in its first run (cause not "
                         "found); it is switched off and positive wave_edges are rejected")
def test_batch_many_tiny_graphs_wave_tier():
    """20,000 graphs of 8 to 200 vertices: the wave tier's workload."""
    import paper_2302_12199_amd as msf
    banner("batch 20k tiny graphs")
    u, v, w, eo, vo = graphgen.batch_gnm(20000, lo=3, hi=7.6, dlo=1, dhi=12, wlo=1, whi=9,
                                         seed=33)
    rm, rt = oracle_batch(u, v, w, eo, vo)
    for wave_edges in (-1, 8192):
        b = make_batch(u, v, w, eo, vo, options=msf.make_batch_options(wave_edges=wave_edges))
        b.launch()
        mask, totals = results(b)
        assert (totals == rt).all() and (mask == rm).all()


def test_batch_bad_graph_flagged_in_every_path():
    import paper_2302_12199_amd as msf
    banner("batch invalid ids")
    u, v, w, eo, vo = graphgen.batch_gnm(40, lo=8, hi=13, seed=22)
    rm, rt = oracle_batch(u, v, w, eo, vo)
    sizes = vo[1:] - vo[:-1]
    big = int(np.argmax(sizes))
    small = int(np.argmin(sizes))
    u = u.copy()
    mid = int(np.argsort(sizes)[len(sizes) // 2])
    u[eo[big]] = sizes[big] + 5           # out of range in a cooperative graph
    u[eo[small] + 1] = sizes[small]       # in an LDS-solved one
    u[eo[mid] + 2] = -1                   # and in one solved in a global slot
    b = make_batch(u, v, w, eo, vo,
                   options=msf.make_batch_options(lds_vertices=1024, wave_edges=-1, coop_edges=int(
                       (eo[big + 1] - eo[big]))))
    b.launch()
    mask, totals = results(b)
    bad = np.zeros(len(rt), bool)
    bad[[big, small, mid]] = True
    assert (totals[bad] == np.uint64(2**64 - 1)).all()
    assert (totals[~bad] == rt[~bad]).all()


def test_batch_unordered_and_ticks():
    banner("batch unordered, ticks")
    u, v, w, eo, vo = graphgen.batch_gnm(120, lo=8, hi=12, dlo=1, dhi=8, wlo=1, whi=7, seed=12)
    rm, rt = oracle_batch(u, v, w, eo, vo)
    b = make_batch(u, v, w, eo, vo, order=None)
    b.launch()
    mask, totals = results(b)
    assert (mask == rm).all() and (totals == rt).all()
    ticks = b.ticks.cpu().numpy().view(np.uint64)
    G = len(rt)
    fin, start0, start = ticks[:G], ticks[G], ticks[G + 1:]
    assert len(start) == G
    # every graph starts after the batch and finishes after it started
    assert (start >= start0).all() and (fin >= start).all()


def test_batch_graph_capture_replays_match_eager():
    import torch
    banner("batch hipGraph replay")
    u, v, w, eo, vo = graphgen.batch_gnm(200, lo=8, hi=12, seed=13)
    rm, rt = oracle_batch(u, v, w, eo, vo)
    b = make_batch(u, v, w, eo, vo)
    b.launch()
    eager = results(b)
    assert (eager[0] == rm).all() and (eager[1] == rt).all()
    b.capture()
    for _ in range(3):
        b.mask.fill_(7)                    # eager work between replays
        b.totals.fill_(0)
        torch.cuda.synchronize()
        b.replay()
        mask, totals = results(b)
        assert (mask == rm).all() and (totals == rt).all()
    b.close()


def test_batch_edge_cases_and_invalid_graph():
    banner("batch edge cases")
    # graph 0: single vertex with self-loops; graph 1: no edges; graph 2: invalid id;
    # graph 3: two vertices, parallel edges; graph 4: ordinary
    gs = [(1, [(0, 0, 5), (0, 0, 1)]), (3, []), (4, [(0, 1, 2), (1, 9, 3)]),
          (2, [(0, 1, 9), (1, 0, 4), (0, 1, 4)]), (5, [(0, 1, 1), (1, 2, 1), (2, 0, 1), (3, 4, 0)])]
    u, v, w, eo, vo = [], [], [], [0], [0]
    for n, es in gs:
        for a, b, c in es:
            u.append(a); v.append(b); w.append(c)
        eo.append(eo[-1] + len(es))
        vo.append(vo[-1] + n)
    u, v, w = np.array(u, np.int32), np.array(v, np.int32), np.array(w, np.uint32)
    eo, vo = np.array(eo, np.int64), np.array(vo, np.int64)
    b = make_batch(u, v, w, eo, vo)
    b.launch()
    mask, totals = results(b)
    assert totals[0] == 0 and totals[1] == 0
    assert totals[2] == np.uint64(2**64 - 1)
    assert totals[3] == 4 and list(mask[eo[3]:eo[4]]) == [0, 1, 0]
    assert totals[4] == 2 and list(mask[eo[4]:eo[5]]) == [1, 1, 0, 1]


def test_batch_autotune_then_correct():
    banner("batch autotune")
    u, v, w, eo, vo = graphgen.batch_gnm(100, lo=8, hi=12, seed=14)
    rm, rt = oracle_batch(u, v, w, eo, vo)
    b = make_batch(u, v, w, eo, vo)
    cfg = b.autotune()
    assert cfg["block"] in (256, 512, 1024) and cfg["ms"] > 0
    b.launch()
    mask, totals = results(b)
    assert (mask == rm).all() and (totals == rt).all()


def test_batch_large_graphs_global_scratch():
    banner("batch large graphs")
    u, v, w, eo, vo = graphgen.batch_gnm(24, lo=15, hi=17.5, seed=15)
    rm, rt = oracle_batch(u, v, w, eo, vo)
    b = make_batch(u, v, w, eo, vo)
    b.launch()
    mask, totals = results(b)
    assert (totals == rt).all() and (mask == rm).all()


def test_batch_sample_of_the_10k_workload():
    """Graphs [4000, 4200) of the 10,000-graph batch workload (the sizes and
    seeds the benchmark uses), default options, against the oracle per graph."""
    banner("batch: slice of the 10k workload")
    u, v, w, eo, vo = graphgen.batch_gnm(10000, lo=8, hi=18, dlo=4, dhi=64, wlo=1,
                                         whi=2**31 - 1, seed=6, first=4000, count=200)
    rm, rt = oracle_batch(u, v, w, eo, vo)
    b = make_batch(u, v, w, eo, vo)
    b.capture()
    b.replay()
    mask, totals = results(b)
    assert (totals == rt).all()
    assert (mask == rm).all()
    b.close()


@pytest.mark.timeout(900)
def test_batch_full_10k_workload_every_graph():
    """The whole 10,000-graph workload (6.5e9 edges) in one captured launch,
    with the default options and with those the autotuner picks for it (what
    the benchmark times); every graph's mask and total against the oracle,
    run on 16 host threads (the oracle's C code releases the GIL)."""
    import concurrent.futures as cf
    import torch
    banner("batch: full 10k workload vs oracle (16 host threads)")
    u, v, w, eo, vo = graphgen.batch_gnm(10000, lo=8, hi=18, dlo=4, dhi=64, wlo=1,
                                         whi=2**31 - 1, seed=6)
    runs = []
    for tune in (False, True):
        b = make_batch(u, v, w, eo, vo)
        if tune:
            banner(f"batch: full 10k workload, autotuned {b.autotune()}")
        b.capture()
        b.replay()
        torch.cuda.synchronize()
        runs.append((b.mask[:int(eo[-1])].cpu().numpy(),
                     b.totals[:b.G].cpu().numpy().view(np.uint64)))
        b.close()
        del b
        torch.cuda.empty_cache()

    def check(lo, hi):
        bad = []
        for g in range(lo, hi):
            a, c = int(eo[g]), int(eo[g + 1])
            mk, t, _ = oracle.kruskal(u[a:c], v[a:c], w[a:c], int(vo[g + 1] - vo[g]))
            if any(t != int(totals[g]) or not np.array_equal(mk, mask[a:c])
                   for mask, totals in runs):
                bad.append(g)
        return bad

    with cf.ThreadPoolExecutor(16) as ex:
        parts = list(ex.map(lambda r: check(*r), [(i, min(i + 50, 10000))
                                                  for i in range(0, 10000, 50)]))
    bad = [g for p in parts for g in p]
    assert not bad, f"{len(bad)} graphs differ, first {bad[:5]}"
