#!/usr/bin/env python3
"""MSF throughput benchmark on one MI355X.

One step = one msf_compute call (the whole hot path: every Borůvka round, or
the Filter-Borůvka recursion with --algo filter) over one synthetic graph that
is already resident in HBM.  Default workload: RMAT, n = 2^24, m = 2^28,
Graph500 probabilities, permuted ids, weights uniform in [1, 255].

Prints ONE JSON line on stdout; progress goes to stderr.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0      # MI355X HBM3E peak, GB/s
DEFAULT_WORKLOAD = "rmat_n2^24_m2^28_w255"
METRIC = "MSF input edges/s (RMAT n=2^24 m=2^28); batched vs plain graphs/s"


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def kernel_source_hash():
    import glob
    h = hashlib.sha256()
    for p in sorted(glob.glob(os.path.join(ROOT, "paper_2302_12199_amd", "csrc", "*"))):
        h.update(open(p, "rb").read())
    return h.hexdigest()[:16]


def load_traffic(kernel, workload):
    """HBM bytes per launch from committed rocprofv3 --pmc summaries, if they
    were taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        data = json.load(open(path))
    except ValueError:
        return None
    rec = data.get(workload, {}).get(kernel)
    if not rec or rec.get("source_hash") != kernel_source_hash():
        return None
    return rec.get("hbm_bytes_per_launch")


def cpu_baseline(u, v, w, n, sample_edges):
    import oracle
    k = min(sample_edges, len(u))
    su, sv, sw = u[:k].copy(), v[:k].copy(), w[:k].copy()
    t = time.perf_counter()
    oracle.kruskal(su, sv, sw, n)
    dt = time.perf_counter() - t
    return {"value": k / dt, "unit": "edges/s", "cores": 1, "kind": "oracle",
            "sample": f"first {k} edges of the same graph (n={n}), single-threaded C Kruskal",
            "seconds": round(dt, 3)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD)
    ap.add_argument("--algo", default="boruvka", choices=["boruvka", "filter"])
    ap.add_argument("--pivot", default="median")
    ap.add_argument("--quantile", type=float, default=0.5)
    ap.add_argument("--cpu-sample", type=int, default=1 << 27,
                    help="edges given to the timed CPU oracle (0 = skip)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: this library runs on one GPU; multi-GPU runs are not part of it "
              f"(asked for --gpus {args.gpus}, WORLD_SIZE={world}).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import graphgen
    import paper_2302_12199_amd as msf

    t = time.perf_counter()
    u, v, w, n = graphgen.workload(args.workload)
    m = len(u)
    log(f"generated {args.workload}: n={n} m={m} in {time.perf_counter() - t:.1f}s")
    dev = torch.device("cuda:0")
    tu, tv, tw = (torch.from_numpy(x.view(np.int32)).to(dev) for x in (u, v, w))
    opts = dict(algo=args.algo, pivot=args.pivot, quantile=args.quantile)
    ws = torch.empty(msf.workspace_bytes(m, n, **opts), dtype=torch.uint8, device=dev)
    mask = torch.empty(m, dtype=torch.uint8, device=dev)
    torch.cuda.synchronize()
    log(f"resident on {torch.cuda.get_device_name(dev)}; workspace {ws.numel() / 2**30:.2f} GiB")

    stats = None
    for i in range(args.warmup):
        _, total, stats = msf.compute(tu, tv, tw, n, workspace=ws, mask_out=mask, **opts)
        log(f"warmup {i}: total={total} rounds={stats['rounds']}")

    msf.profile_reset()
    msf.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        _, total, stats = msf.compute(tu, tv, tw, n, workspace=ws, mask_out=mask, **opts)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    msf.profile_enable(False)
    prof = msf.profile_read()
    ms_per_step = (t1 - t0) * 1000.0 / args.steps
    log(f"timed {args.steps} steps: {ms_per_step:.3f} ms/step total={total}")

    dom = max(prof, key=lambda k: prof[k]["ms"]) if prof else None
    roofline = None
    if dom:
        p = prof[dom]
        achieved = p["bytes"] / (p["ms"] / 1000.0) / 1e9
        traffic = load_traffic(dom, args.workload)
        roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1),
                    "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4),
                    "traffic": traffic,
                    "launch_ms": round(p["ms"] / p["launches"], 4),
                    "algorithmic_bytes_per_launch": p["bytes"] / p["launches"]}
    kernels = {k: {"ms_per_step": round(x["ms"] / args.steps, 4),
                   "launches_per_step": x["launches"] / args.steps,
                   "GBps": round(x["bytes"] / (x["ms"] / 1000.0) / 1e9, 1) if x["ms"] > 0 else None}
               for k, x in sorted(prof.items(), key=lambda kv: -kv[1]["ms"])}

    cpu = None
    if args.cpu_sample > 0:
        cpu = cpu_baseline(u, v, w, n, args.cpu_sample)
        log(f"cpu oracle: {cpu['value']:.3e} edges/s over {cpu['sample']}")

    out = {
        "metric": METRIC, "value": m / (ms_per_step / 1000.0), "unit": "edges/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": args.workload, "n": int(n), "m": int(m), "algo": args.algo,
                   "pivot": args.pivot if args.algo == "filter" else None},
        "roofline": roofline, "cpu_baseline": cpu,
        "detail": {"rounds": stats["rounds"], "round_live": stats["round_live"],
                   "round_edges": stats["round_edges"], "msf_edges": stats["msf_edges"],
                   "total_weight": stats["total_weight"], "kernels": kernels},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
