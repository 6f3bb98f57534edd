"""msf_compute_noalloc, the entry point that allocates nothing (its workspace
is the library's static per-GPU scratch array), against msf_compute on the
same inputs, through the C ABI (needs a GPU).

Bar: integer work, so the masks are equal byte for byte and the totals and
per-round counts equal; the oracle checks the first call as well."""
import ctypes

import numpy as np
import pytest

import graphgen
import oracle
from gpu_util import banner, to_dev

pytestmark = pytest.mark.gpu


def run_both(msf, u, v, w, n, **opts):
    import torch
    tu, tv, tw = to_dev(u, v, w)
    m = len(u)
    ref_mask, ref_total, ref_stats = msf.compute(tu, tv, tw, n, **opts)
    ref_mask = ref_mask.cpu().numpy()
    # a mask buffer holding stale ones: the call must clear it itself
    out = torch.ones(max(m, 1), dtype=torch.uint8, device=tu.device)[:m]
    mask, total, stats = msf.compute_noalloc(tu, tv, tw, n, mask_out=out, **opts)
    torch.cuda.synchronize()
    got = mask.cpu().numpy()
    assert (got == ref_mask).all(), f"masks differ at {np.nonzero(got != ref_mask)[0][:10]}"
    assert total == ref_total
    for k in ("msf_edges", "rounds", "round_live", "round_edges", "round_found", "levels",
              "splits"):
        assert stats[k] == ref_stats[k], k
    return got, total


@pytest.mark.parametrize("algo", ["boruvka", "filter"])
def test_noalloc_matches_msf_compute_twice_second_smaller(algo):
    import paper_2302_12199_amd as msf
    opts = dict(algo=algo, min_split_edges=1 << 14) if algo == "filter" else {}
    # first call: GNM n = 2^16, m = 2^20 (the small configuration), then a
    # smaller RMAT graph whose state lands on what the first call left behind
    u, v, w = graphgen.gnm(1 << 16, 1 << 20, 1, 2**31 - 1, seed=1)
    banner(f"noalloc {algo}: gnm n=2^16 m=2^20")
    got, total = run_both(msf, u, v, w, 1 << 16, **opts)
    rm, rt, _ = oracle.kruskal(u, v, w, 1 << 16)
    assert (got == rm).all() and total == rt
    u2, v2, w2 = graphgen.rmat(13, 50000, seed=5, wlo=1, whi=255)
    banner(f"noalloc {algo}: rmat n=2^13 m=50000")
    got2, total2 = run_both(msf, u2, v2, w2, 1 << 13, **opts)
    rm2, rt2, _ = oracle.kruskal(u2, v2, w2, 1 << 13)
    assert (got2 == rm2).all() and total2 == rt2


def test_noalloc_rejects_graphs_beyond_the_scratch():
    import paper_2302_12199_amd as msf
    m, n = 4 << 20, 1 << 20
    assert msf.workspace_bytes(m, n) > msf.NOALLOC_SCRATCH_BYTES
    total = ctypes.c_uint64(0)
    rc = msf.library().msf_compute_noalloc(0x1000, 0x1000, 0x1000, m, n, 0x1000,
                                           ctypes.byref(total), None, None, None)
    assert rc == msf.EWORKSPACE
    assert b"static scratch" in msf.library().msf_last_error()
