"""The graphs whose MSF is known by construction (tests/known_msf.py, used at
the library's maximum sizes on the GPU) checked on the CPU at small sizes:
the stated mask and total against the oracle's Kruskal, and the certificate
checker on the stated mask."""
import math

import numpy as np
import pytest

import oracle
from known_msf import STRIDE, known_msf_graph


@pytest.mark.parametrize("local", [False, True])
@pytest.mark.parametrize("m,n,seed", [(70001, 3000, 1), (200003, 50000, 2), (40961, 20000, 3)])
def test_known_msf_matches_oracle(m, n, seed, local):
    assert math.gcd(STRIDE, m) == 1
    u, v, w, exp, total, count = known_msf_graph(m, n, device="cpu", seed=seed, local=local)
    un, vn = u.numpy(), v.numpy()
    wn = w.numpy().view(np.uint32)
    mask, t, _ = oracle.kruskal(un, vn, wn, n)
    assert np.array_equal(mask, exp.numpy())
    assert t == total and int(mask.sum()) == count
    assert oracle.check(un, vn, wn, n, exp.numpy())[0] == 0
    if local:   # ids rise along the edge list: the locality the window kernels exploit
        d = np.abs(un.astype(np.int64) - vn.astype(np.int64))
        assert np.mean(d < 2**14) > 0.9


def test_known_msf_has_copies_won_both_ways():
    """Some copies win by weight, some by position, some lose: every branch of
    the construction is exercised."""
    m, n = 70001, 3000
    u, v, w, exp, _, _ = known_msf_graph(m, n, device="cpu", seed=7)
    import torch
    k = torch.arange(1, n, dtype=torch.int64)
    sel = k % 4 == 0
    pos = (k[sel] * STRIDE) % m
    q = ((k[sel] + n) * STRIDE) % m
    wins = exp[q] == 1
    assert wins.any() and (~wins).any()
    lighter = (w[q] < w[pos]) & wins
    by_position = (w[q] == w[pos]) & wins
    assert lighter.any() and by_position.any()
    assert torch.equal(exp[pos] + exp[q], torch.ones_like(exp[q]))


def test_known_msf_rejects_bad_sizes():
    for m, n in ((199, 100), (2 * STRIDE, 100), (2**32 - 1, 1)):   # m < 2n, shared factor, n < 2
        with pytest.raises(ValueError):
            known_msf_graph(m, n, device="cpu", seed=1)
