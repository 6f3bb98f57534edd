"""Training of the Filter-Borůvka pivot network.

The paper splits each edge set at the median of a random sample (Alg. 2);
any split point gives the same forest, so the quantile only changes run time.
This module builds the network's data set and trains it:

  sweep  - for generated graphs (several families, sizes and densities) time
           msf_compute(algo=filter) at every quantile of a log-spaced grid and
           record the top split's sample features;
  train  - fit the network (the library's own FP32/BF16 forward and backward
           kernels, Adam) to the soft minimum of each graph's timing curve;
  eval   - load the trained network and time it against the median pivot and
           the best swept quantile on held-out graphs (regret).

Usage (needs the GPU):
  python -m paper_2302_12199_amd.pivot_train all --out DIR [--quick]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

Q_GRID = [2.0**-10, 2.0**-8, 2.0**-6, 2.0**-4, 0.125, 0.25, 0.375, 0.5, 0.625, 0.75, 0.85,
          0.9, 0.95]


def log(*a):
    print("[pivot]", *a, file=sys.stderr, flush=True)


def graph_specs(quick=False):
    """(name, family, params, seed) of the sweep graphs."""
    specs = []
    ms = [1 << 22, 1 << 24] if quick else [1 << 22, 1 << 23, 1 << 24, 1 << 25, 1 << 26]
    degs = [16, 64] if quick else [8, 16, 32, 64, 128, 256]
    seeds = [1] if quick else [1, 2]
    for m in ms:
        for d in degs:
            n = max(1 << 10, (2 * m) // d)
            for s in seeds:
                specs.append((f"gnm_n{n}_m{m}_s{s}", "gnm", dict(n=n, m=m), s))
                scale = max(10, int(round(math.log2(n))))
                specs.append((f"rmat_s{scale}_m{m}_w31_s{s}", "rmat",
                              dict(scale=scale, m=m, whi=2**31 - 1), s))
                if d in (16, 64, 128):
                    specs.append((f"rmat_s{scale}_m{m}_w255_s{s}", "rmat",
                                  dict(scale=scale, m=m, whi=255), s))
    if not quick:
        for side in (1024, 2048):
            specs.append((f"grid_{side}", "grid", dict(side=side), 1))
        for lg in (20, 22):
            specs.append((f"rgg_n2^{lg}_d32", "rgg", dict(n=1 << lg, deg=32), 1))
    return specs


def make_graph(family, p, seed):
    import graphgen
    if family == "gnm":
        u, v, w = graphgen.gnm(p["n"], p["m"], 1, 2**31 - 1, seed)
        return u, v, w, p["n"]
    if family == "rmat":
        u, v, w = graphgen.rmat(p["scale"], p["m"], wlo=1, whi=p["whi"], seed=seed + 10)
        return u, v, w, 1 << p["scale"]
    if family == "grid":
        u, v, w = graphgen.grid(p["side"], p["side"], keep=0.8, wlo=1, whi=2**20, seed=seed)
        return u, v, w, p["side"] * p["side"]
    if family == "rgg":
        r = graphgen.rgg_radius(p["n"], p["deg"])
        u, v, w = graphgen.rgg2d(p["n"], r, seed=seed)
        return u, v, w, p["n"]
    raise ValueError(family)


class Runner:
    """Resident graph + workspace; times filter runs at a given pivot rule."""

    def __init__(self, u, v, w, n):
        import torch

        import paper_2302_12199_amd as msf
        self.msf, self.torch = msf, torch
        dev = torch.device("cuda:0")
        self.t = [torch.from_numpy(np.ascontiguousarray(x).view(np.int32)).to(dev)
                  for x in (u, v, w)]
        self.n, self.m = n, len(u)
        self.ws = torch.empty(msf.workspace_bytes(self.m, n, algo="filter"), dtype=torch.uint8,
                              device=dev)
        self.mask = torch.empty(max(self.m, 1), dtype=torch.uint8, device=dev)

    def run(self, **opts):
        tu, tv, tw = self.t
        return self.msf.compute(tu, tv, tw, self.n, workspace=self.ws, mask_out=self.mask,
                                algo="filter", **opts)

    def time(self, reps=3, **opts):
        self.run(**opts)
        ts = []
        for _ in range(reps):
            self.torch.cuda.synchronize()
            t = time.perf_counter()
            _, total, st = self.run(**opts)
            self.torch.cuda.synchronize()
            ts.append(time.perf_counter() - t)
        return float(np.median(ts)), total, st


def sweep(specs, reps, out_path):
    rows = []
    for name, fam, p, seed in specs:
        t0 = time.perf_counter()
        u, v, w, n = make_graph(fam, p, seed)
        r = Runner(u, v, w, n)
        tmed, total, st = r.time(reps, pivot="median")
        if st["levels"] == 0:
            log(f"{name}: no split (sparse), skipped")
            continue
        times = []
        for q in Q_GRID:
            tq, tot_q, _ = r.time(reps, pivot="quantile", quantile=q)
            if tot_q != total:
                raise RuntimeError(f"{name}: total differs at q={q}")
            times.append(tq)
        rows.append({"name": name, "family": fam, "n": int(n), "m": int(len(u)),
                     "features": st["top_features"], "q_grid": Q_GRID, "times": times,
                     "median_time": tmed, "levels": st["levels"]})
        best = int(np.argmin(times))
        log(f"{name}: median {tmed * 1e3:.2f} ms, best q={Q_GRID[best]:.4g} "
            f"{times[best] * 1e3:.2f} ms ({time.perf_counter() - t0:.1f}s)")
        del r
        json.dump({"q_grid": Q_GRID, "rows": rows}, open(out_path, "w"))
    return rows


def soft_target(q_grid, times, tau=0.03):
    """Logit of the soft-argmin quantile: weights exp(-(t/tmin - 1)/tau)."""
    t = np.asarray(times)
    wts = np.exp(-(t / t.min() - 1.0) / tau)
    lq = np.log(np.asarray(q_grid)) - np.log1p(-np.asarray(q_grid))
    return float((wts * lq).sum() / wts.sum())


def interp_time(q_grid, times, q):
    lq = np.log(np.asarray(q_grid)) - np.log1p(-np.asarray(q_grid))
    x = math.log(q) - math.log1p(-q)
    return float(np.interp(x, lq, times))


def split_rows(rows):
    """Held-out set: every row whose name hashes into the last quarter."""
    import zlib
    tr, te = [], []
    for r in rows:
        (te if zlib.crc32(r["name"].encode()) % 4 == 3 else tr).append(r)
    return tr, te


def train(rows, steps=3000, lr=2e-3, seed=0, bf16=True):
    import torch

    import paper_2302_12199_amd as msf
    x = np.array([r["features"] for r in rows], np.float32)
    t = np.array([soft_target(r["q_grid"], r["times"]) for r in rows], np.float32)
    dev = torch.device("cuda:0")
    tx, tt = torch.from_numpy(x).to(dev), torch.from_numpy(t).to(dev)
    p = torch.from_numpy(msf.init_pivot_params(seed)).to(dev)
    m, v = torch.zeros_like(p), torch.zeros_like(p)
    hist = []
    for step in range(1, steps + 1):
        g, loss = msf.mlp_grad(p, tx, tt, bf16=bf16)
        msf.mlp_adam(p, g, m, v, step, lr=lr)
        if step % 500 == 0 or step == 1:
            hist.append((step, float(loss.item())))
    return p.cpu().numpy(), t, hist


def predict_q(params, feats):
    import torch

    import paper_2302_12199_amd as msf
    x = torch.from_numpy(np.asarray(feats, np.float32).reshape(-1, 16)).cuda()
    z = msf.mlp_forward(torch.from_numpy(params).cuda(), x, bf16=True).cpu().numpy()
    q = 1.0 / (1.0 + np.exp(-z.astype(np.float64)))
    return np.clip(q, 2.0**-10, 1 - 2.0**-10)


def evaluate(specs, model_path, reps, rows_by_name):
    """Times the loaded network against the median pivot (and the best swept
    quantile where the graph was swept) on freshly generated graphs."""
    import paper_2302_12199_amd as msf
    msf.load_pivot_model(model_path)
    out = []
    try:
        for name, fam, p, seed in specs:
            u, v, w, n = make_graph(fam, p, seed)
            r = Runner(u, v, w, n)
            tmed, total, _ = r.time(reps, pivot="median")
            tnet, total_net, st = r.time(reps, pivot="mlp")
            if total_net != total:
                raise RuntimeError(f"{name}: total differs with the network pivot")
            rec = {"name": name, "t_median": tmed, "t_net": tnet, "q_net": st["pivot_q_used"],
                   "speedup_vs_median": tmed / tnet}
            sw = rows_by_name.get(name)
            if sw:
                rec["t_best_swept"] = min(sw["times"])
                rec["regret_vs_best"] = tnet / rec["t_best_swept"] - 1.0
            log(f"eval {name}: median {tmed * 1e3:.2f} ms, network q={rec['q_net']:.3f} "
                f"{tnet * 1e3:.2f} ms")
            out.append(rec)
            del r
    finally:
        msf.clear_pivot_model()
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("cmd", choices=["sweep", "train", "all"])
    ap.add_argument("--out", default="gpurun_out/pivot")
    ap.add_argument("--quick", action="store_true")
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--steps", type=int, default=3000)
    args = ap.parse_args(argv)
    os.makedirs(args.out, exist_ok=True)
    sweep_path = os.path.join(args.out, "pivot_sweep.json")
    if args.cmd in ("sweep", "all"):
        sweep(graph_specs(args.quick), args.reps, sweep_path)
    if args.cmd in ("train", "all"):
        import paper_2302_12199_amd as msf
        rows = json.load(open(sweep_path))["rows"]
        tr, te = split_rows(rows)
        log(f"training on {len(tr)} graphs, {len(te)} held out")
        params, _, hist = train(tr, steps=args.steps)
        for s, l in hist:
            log(f"step {s}: loss {l:.4f}")
        open(os.path.join(args.out, "pivot_mlp.bin"), "wb").write(msf.model_blob(params))
        report = {"train_loss": hist, "graphs": []}
        for split, rs in (("train", tr), ("heldout", te)):
            if not rs:
                continue
            qs = predict_q(params, [r["features"] for r in rs])
            for r, q in zip(rs, qs):
                best = float(min(r["times"]))
                tq = interp_time(r["q_grid"], r["times"], float(q))
                report["graphs"].append({
                    "name": r["name"], "set": split, "q_pred": float(q),
                    "q_best": r["q_grid"][int(np.argmin(r["times"]))],
                    "t_best": best, "t_median": r["median_time"], "t_pred_interp": tq,
                    "regret_vs_best": tq / best - 1.0, "gain_vs_median": r["median_time"] / tq})
        for split in ("train", "heldout"):
            g = [x for x in report["graphs"] if x["set"] == split]
            if g:
                report[split] = {
                    "graphs": len(g),
                    "mean_regret_vs_best": float(np.mean([x["regret_vs_best"] for x in g])),
                    "geomean_gain_vs_median": float(np.exp(np.mean(
                        [math.log(x["gain_vs_median"]) for x in g])))}
                log(f"{split}: {report[split]}")
        by_name = {r["name"]: r for r in rows}
        held = [sp for sp in graph_specs(args.quick) if sp[0] in {r["name"] for r in te}]
        held.append(("rmat_s22_m268435456_w31_s1", "rmat", dict(scale=22, m=1 << 28,
                                                               whi=2**31 - 1), 1))
        report["measured"] = evaluate(held, os.path.join(args.out, "pivot_mlp.bin"), args.reps,
                                      by_name)
        json.dump(report, open(os.path.join(args.out, "pivot_report.json"), "w"), indent=1)


if __name__ == "__main__":
    main()
