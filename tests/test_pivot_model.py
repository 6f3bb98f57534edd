"""The shipped pivot network: format, and what it gains over the median pivot
on the timing sweep it was trained from (timings measured on an MI355X by
paper_2302_12199_amd/pivot_train.py; held-out graphs were not trained on)."""
import json
import math
import os

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
DATA = os.path.join(ROOT, "paper_2302_12199_amd", "data")


def _params():
    from oracle import mlp_ref
    blob = open(os.path.join(DATA, "pivot_mlp.bin"), "rb").read()
    hdr = np.frombuffer(blob[:16], np.uint32)
    assert list(hdr) == [0x5046534D, 1, mlp_ref.IN, mlp_ref.H]
    p = np.frombuffer(blob[16:], np.float32).astype(np.float64)
    assert p.shape == (mlp_ref.P,) and np.isfinite(p).all()
    return p


def _interp(q_grid, times, q):
    lq = np.log(np.asarray(q_grid)) - np.log1p(-np.asarray(q_grid))
    return float(np.interp(math.log(q) - math.log1p(-q), lq, times))


def test_shipped_model_gains_over_median_on_held_out_graphs():
    import zlib
    from oracle import mlp_ref
    p = _params()
    sweep = json.load(open(os.path.join(DATA, "pivot_sweep.json")))
    rows = [r for r in sweep["rows"] if zlib.crc32(r["name"].encode()) % 4 == 3]
    assert len(rows) >= 20
    feats = np.array([r["features"] for r in rows], np.float64)
    z, _ = mlp_ref.forward(p, feats, bf=True)
    q = mlp_ref.quantile(z)
    gains, regrets = [], []
    for r, qq in zip(rows, q):
        t_net = _interp(r["q_grid"], r["times"], float(qq))
        gains.append(r["median_time"] / t_net)
        regrets.append(t_net / min(r["times"]) - 1.0)
    geo = math.exp(np.mean(np.log(gains)))
    assert geo >= 1.05, geo                 # faster than the median pivot overall
    assert np.median(regrets) <= 0.10       # close to the best swept quantile


def test_shipped_model_report_measured_no_slower_than_median_overall():
    rep = json.load(open(os.path.join(DATA, "pivot_report.json")))
    meas = rep["measured"]
    sp = [m["speedup_vs_median"] for m in meas]
    assert math.exp(np.mean(np.log(sp))) >= 1.0
    c4 = [m for m in meas if m["name"].startswith("rmat_s22_m268435456")]
    assert c4 and c4[0]["speedup_vs_median"] >= 1.0
