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


BATCH_WORKLOAD = "batch_gnm_10k_n2^8..2^18_deg4..64"


def run_batch(args):
    """Batched solve of the 10,000-graph GNM batch (n log-uniform in
    [2^8, 2^18], average degree uniform in [4, 64], w uniform in [1, 2^31)):
    one hipGraph-captured persistent launch per step, against a loop of
    per-graph msf_compute calls on a sample of the same batch."""
    import numpy as np
    import torch

    import graphgen
    import paper_2302_12199_amd as msf

    G = args.graphs
    t = time.perf_counter()
    u, v, w, eo, vo = graphgen.batch_gnm(G, lo=8, hi=18, dlo=4, dhi=64, wlo=1, whi=2**31 - 1,
                                         seed=6)
    m = int(eo[-1])
    log(f"generated {G} graphs, {m} edges in {time.perf_counter() - t:.1f}s")
    dev = torch.device("cuda:0")
    tu, tv, tw = (torch.from_numpy(x.view(np.int32)).to(dev) for x in (u, v, w))
    b = msf.Batch(tu, tv, tw, eo, vo)
    torch.cuda.synchronize()
    tuned = b.autotune() if args.autotune else None
    if tuned:
        log(f"autotuned: {tuned}")
    b.capture()
    for _ in range(args.warmup):
        b.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        b.replay()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_batch = (t1 - t0) * 1000.0 / args.steps
    ticks = b.ticks.cpu().numpy().view(np.uint64).astype(np.float64)
    khz = msf.wall_clock_khz()
    lat_ms = (ticks[:-1] - ticks[-1]) / khz if khz else np.zeros(G)
    log(f"batched: {ms_batch:.2f} ms per batch, {G / ms_batch * 1000:.0f} graphs/s")

    # plain per-graph calls on a sample of the batch (same graphs, same order)
    k = min(args.plain_sample, G)
    max_e = int((eo[1:k + 1] - eo[:k]).max())
    max_n = int((vo[1:k + 1] - vo[:k]).max())
    ws = torch.empty(msf.workspace_bytes(max_e, max_n), dtype=torch.uint8, device=dev)
    mk = torch.empty(max(max_e, 1), dtype=torch.uint8, device=dev)
    torch.cuda.synchronize()
    per = []
    t0 = time.perf_counter()
    for g in range(k):
        a, c = int(eo[g]), int(eo[g + 1])
        tg = time.perf_counter()
        msf.compute(tu[a:c], tv[a:c], tw[a:c], int(vo[g + 1] - vo[g]), workspace=ws,
                    mask_out=mk[:c - a])
        per.append(time.perf_counter() - tg)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    plain_gps = k / (t1 - t0)
    batch_gps = G / (ms_batch / 1000.0)
    log(f"plain: {plain_gps:.0f} graphs/s over {k} graphs")
    out = {
        "metric": "batched graphs/s (10,000 GNM graphs) vs per-graph plain calls",
        "value": batch_gps, "unit": "graphs/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_batch, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": BATCH_WORKLOAD, "graphs": G, "edges": m},
        "batched_edges_per_s": m / (ms_batch / 1000.0),
        "plain_graphs_per_s": plain_gps, "plain_sample": k,
        "speedup_vs_plain": batch_gps / plain_gps,
        "latency_ms": {"p50": float(np.percentile(lat_ms, 50)),
                       "p99": float(np.percentile(lat_ms, 99)),
                       "max": float(lat_ms.max())},
        "plain_service_ms": {"p50": 1000 * float(np.percentile(per, 50)),
                             "p99": 1000 * float(np.percentile(per, 99))},
        "autotuned": tuned,
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD)
    ap.add_argument("--algo", default="boruvka", choices=["boruvka", "filter"])
    ap.add_argument("--pivot", default="median")
    ap.add_argument("--quantile", type=float, default=0.5)
    ap.add_argument("--model", default=None, help="pivot network file (--pivot mlp)")
    ap.add_argument("--no-alternative", action="store_true",
                    help="with --algo boruvka: skip timing Filter-Borůvka on the same graph")
    ap.add_argument("--no-pivot-compare", action="store_true",
                    help="with --pivot mlp: skip the timed median-pivot comparison")
    ap.add_argument("--cpu-sample", type=int, default=1 << 27,
                    help="edges given to the timed CPU oracle (0 = skip)")
    ap.add_argument("--graphs", type=int, default=10000, help="batch workload: graphs")
    ap.add_argument("--plain-sample", type=int, default=300,
                    help="batch workload: graphs timed with per-graph calls")
    ap.add_argument("--autotune", action="store_true", help="batch workload: autotune first")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (calibrates byte counters)")
    args = ap.parse_args()

    if args.copy_calibration:
        import torch
        a = torch.empty(1 << 30, dtype=torch.uint8, device="cuda:0").fill_(1)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        log("copied 1 GiB three times")
        return

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: this library runs on one GPU; multi-GPU runs are not part of it "
              f"(asked for --gpus {args.gpus}, WORLD_SIZE={world}).", file=sys.stderr)
        sys.exit(2)

    if args.workload == BATCH_WORKLOAD:
        return run_batch(args)

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
    if args.algo == "filter" and args.pivot == "mlp":
        msf.load_pivot_model(args.model)        # default: the shipped network
        log(f"pivot network loaded from {args.model or msf.DEFAULT_MODEL}")
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

    pivot_cmp = None
    if args.algo == "filter" and args.pivot == "mlp" and not args.no_pivot_compare:
        # the same graph with the sampled-median pivot, for comparison
        mopts = dict(opts, pivot="median")
        for _ in range(args.warmup):
            msf.compute(tu, tv, tw, n, workspace=ws, mask_out=mask, **mopts)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        for _ in range(args.steps):
            _, mtotal, _ = msf.compute(tu, tv, tw, n, workspace=ws, mask_out=mask, **mopts)
        torch.cuda.synchronize()
        med_ms = (time.perf_counter() - t2) * 1000.0 / args.steps
        if mtotal != total:
            raise RuntimeError("median-pivot run gave a different total")
        pivot_cmp = {"median_ms_per_step": round(med_ms, 4), "network_q": stats["pivot_q_used"],
                     "speedup_vs_median": round(med_ms / ms_per_step, 4)}
        log(f"median pivot: {med_ms:.3f} ms/step; network q={stats['pivot_q_used']:.4f}")

    dom = max(prof, key=lambda k: prof[k]["ms"]) if prof else None
    roofline = None
    if dom:
        p = prof[dom]
        achieved = p["bytes"] / (p["ms"] / 1000.0) / 1e9
        traffic = load_traffic(dom, args.workload)
        launch_ms = p["ms"] / p["launches"]
        roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1),
                    "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4),
                    "traffic": traffic,
                    "launch_ms": round(launch_ms, 4),
                    "algorithmic_bytes_per_launch": p["bytes"] / p["launches"]}
        if traffic:
            # measured HBM bytes (random gathers move whole 128-byte lines) over the same time
            tg = traffic / (launch_ms / 1000.0) / 1e9
            roofline["traffic_GBps"] = round(tg, 1)
            roofline["traffic_frac"] = round(tg / PEAK_HBM_GBS, 4)
    kernels = {k: {"ms_per_step": round(x["ms"] / args.steps, 4),
                   "launches_per_step": x["launches"] / args.steps,
                   "GBps": round(x["bytes"] / (x["ms"] / 1000.0) / 1e9, 1) if x["ms"] > 0 else None}
               for k, x in sorted(prof.items(), key=lambda kv: -kv[1]["ms"])}

    alt = None
    if args.algo == "boruvka" and not args.no_alternative:
        # the same graph through Filter-Borůvka with the shipped pivot network
        # (reported beside the configured plain Borůvka, not as the value)
        msf.load_pivot_model()
        fopts = dict(algo="filter", pivot="mlp")
        fws = torch.empty(msf.workspace_bytes(m, n, **fopts), dtype=torch.uint8, device=dev)
        for _ in range(args.warmup):
            msf.compute(tu, tv, tw, n, workspace=fws, mask_out=mask, **fopts)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        for _ in range(args.steps):
            _, ftotal, fst = msf.compute(tu, tv, tw, n, workspace=fws, mask_out=mask, **fopts)
        torch.cuda.synchronize()
        fms = (time.perf_counter() - t2) * 1000.0 / args.steps
        msf.clear_pivot_model()
        del fws
        if ftotal != total:
            raise RuntimeError("Filter-Borůvka gave a different total")
        alt = {"algo": "filter", "pivot": "mlp", "network_q": fst["pivot_q_used"],
               "ms_per_step": round(fms, 4), "edges_per_s": m / (fms / 1000.0)}
        log(f"filter + pivot network: {fms:.3f} ms/step (q={fst['pivot_q_used']:.3f})")

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
        "roofline": roofline, "cpu_baseline": cpu, "pivot_vs_median": pivot_cmp,
        "same_graph_filter_boruvka": alt,
        "detail": {"rounds": stats["rounds"], "round_live": stats["round_live"],
                   "round_edges": stats["round_edges"], "msf_edges": stats["msf_edges"],
                   "total_weight": stats["total_weight"], "kernels": kernels},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
