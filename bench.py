#!/usr/bin/env python3
"""MSF throughput benchmark on one MI355X.

One step = one msf_compute call (the whole hot path: every Borůvka round, or
the Filter-Borůvka recursion) over one synthetic graph that is already
resident in HBM.  The headline workload is RMAT, n = 2^24, m = 2^28, Graph500
probabilities, permuted ids, weights uniform in [1, 255], plain Borůvka.

After the headline the same run measures the other workloads (fewer steps):
GNM n = 2^16 m = 2^20; the 4096 x 4096 grid with constant and with [1, 255]
weights; the 2D random geometric graph n = 2^24 of average degree 8; RMAT
n = 2^22 m = 2^28 through Filter-Borůvka with the pivot network against the
sampled-median pivot; and the batch of 10,000 GNM graphs, one captured
persistent launch against per-graph calls.  `--no-extras` skips them.

Timed steps run with the library's kernel profiler off; the per-kernel table
comes from a separate profiled pass over the same workload.

Prints ONE JSON line on stdout; progress goes to stderr.
"""
import argparse
import hashlib
import re
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0      # MI355X HBM3E peak, GB/s
DEFAULT_WORKLOAD = "rmat_n2^24_m2^28_w255"
BATCH_WORKLOAD = "batch_gnm_10k_n2^8..2^18_deg4..64"
METRIC = "MSF input edges/s (RMAT n=2^24 m=2^28); batched vs plain graphs/s"

# Source files of each kernel family: a stored counter reading stays valid
# while these are unchanged.
CSRC = os.path.join(ROOT, "paper_2302_12199_amd", "csrc")
COMMON = ["common.h", "prim.h", "launch.h"]
FAMILY_SOURCES = {
    "bucket_pass": ["bucket.hip", "bucket.h"], "bucket_min": ["bucket.hip", "bucket.h"],
    "bucket_scatter": ["bucket.hip", "bucket.h"], "bucket_label": ["bucket.hip", "bucket.h"],
    "bucket_index": ["bucket.hip", "bucket.h"], "pass": ["boruvka.hip"],
    "compact": ["boruvka.hip"], "hook": ["boruvka.hip"], "minedge_r0": ["boruvka.hip"],
    "scan_roots": ["boruvka.hip"], "label": ["boruvka.hip"], "jump": ["boruvka.hip"],
    "tail": ["tail.hip"], "filter": ["filter.hip"], "partition": ["filter.hip"],
    "sample": ["filter.hip", "mlp.h"], "batch": ["batch.hip", "batch.h"],
}


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def _code_only(text):
    """Source text without comments and blank space: an edited comment does not
    change the code a counter reading was taken on."""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def family_source_hash(family):
    h = hashlib.sha256()
    for name in sorted(set(FAMILY_SOURCES.get(family, []) + COMMON)):
        p = os.path.join(CSRC, name)
        if os.path.exists(p):
            h.update(name.encode())
            h.update(_code_only(open(p, encoding="utf-8").read()).encode())
    return h.hexdigest()[:16]


def load_traffic(kernel, workload):
    """HBM bytes per launch from committed rocprofv3 --pmc readings, if they
    were taken on the kernel family's current sources; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        data = json.load(open(path))
    except ValueError:
        return None
    rec = data.get(workload, {}).get(kernel)
    if not rec or rec.get("source_hash") != family_source_hash(kernel):
        return None
    return rec.get("hbm_bytes_per_launch")


# ------------------------------------------------------- algorithmic bytes

def round_bytes(stats, m0):
    """Bytes the Borůvka rounds must move (per round r, from the counts the
    call reports): m_r edges and n_r vertex labels entering round r, m'_r =
    m_{r+1} edges surviving its relabelling.
      lightest edge       16 B per edge read (12 B in round 0: the input),
                          16 B per vertex (best[] set and read)
      hook + MSF mark     20 B per vertex (parent written, endpoints and a
                          label gathered)
      pointer jumping     12 B per vertex per sweep (one sweep counted)
      contraction         12 B per vertex
      relabel + compact   16 B per edge read (12 B in round 0) + 8 B of label
                          gathers per edge + 16 B per surviving edge written
    plus the output mask, 1 B per input edge.  Returns (total, per round)."""
    me = stats["round_edges"]
    nv = stats["round_vertices"]
    per = []
    for r in range(len(me)):
        m_r, n_r = me[r], nv[r]
        m_next = me[r + 1] if r + 1 < len(me) else 0
        rd = 12 if r == 0 else 16
        b = rd * m_r + 16 * n_r + 20 * n_r + 12 * n_r + 12 * n_r + (rd + 8) * m_r + 16 * m_next
        per.append(b)
    return sum(per) + m0, per


def dominant_launch_bytes(family, stats):
    """Algorithmic bytes of one launch of the dominant family, from the same
    per-step figures: the bucketed relabelling pass of round 0 performs round
    0's relabel + compact (12 B read + 8 B gathered per input edge, 16 B per
    surviving edge written) and round 1's lightest-edge search fused into it
    (16 B per round-1 edge, 16 B per round-1 vertex).  None for families this
    model does not cover."""
    me, nv = stats["round_edges"], stats["round_vertices"]
    if family == "bucket_pass" and len(me) >= 2:
        return (12 + 8) * me[0] + 16 * me[1] + 16 * me[1] + 16 * nv[1]
    return None


# ------------------------------------------------------------ single graph

def timed(fn, steps, warmup):
    import torch
    out = None
    for _ in range(warmup):
        out = fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        out = fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1000.0 / steps, out


def kernel_table(msf, fn, steps):
    """Per-family event times from a separate profiled pass."""
    import torch
    torch.cuda.synchronize()
    msf.profile_reset()
    msf.profile_enable(True)
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    msf.profile_enable(False)
    prof = msf.profile_read()
    msf.profile_reset()
    return prof


def measure_graph(msf, tu, tv, tw, n, workload, steps, warmup, prof_steps, **opts):
    """Timed steps (profiler off), then a profiled pass.  Returns a record."""
    import torch
    m = tu.numel()
    ws = torch.empty(max(msf.workspace_bytes(m, n, **opts), 1), dtype=torch.uint8,
                     device=tu.device)
    mask = torch.empty(max(m, 1), dtype=torch.uint8, device=tu.device)[:m]

    def step():
        return msf.compute(tu, tv, tw, n, workspace=ws, mask_out=mask, **opts)

    ms, (_, total, stats) = timed(step, steps, warmup)
    prof = kernel_table(msf, step, prof_steps)
    del ws
    kernels = {k: {"ms_per_step": round(x["ms"] / prof_steps, 4),
                   "launches_per_step": x["launches"] / prof_steps,
                   "avg_launch_ms": round(x["ms"] / max(x["launches"], 1), 4),
                   "own_GBps": round(x["bytes"] / (x["ms"] / 1000.0) / 1e9, 1)
                   if x["ms"] > 0 else None}
               for k, x in sorted(prof.items(), key=lambda kv: -kv[1]["ms"])}
    alg_total, _ = round_bytes(stats, m)
    rec = {"workload": workload, "n": int(n), "m": int(m), "ms_per_step": round(ms, 4),
           "edges_per_s": m / (ms / 1000.0), "total_weight": total,
           "msf_edges": stats["msf_edges"], "rounds": stats["rounds"],
           "round_edges": stats["round_edges"], "round_vertices": stats["round_vertices"],
           "kernels": kernels, "_prof": prof, "_stats": stats}
    if opts.get("algo", "boruvka") == "boruvka":
        rec["algorithmic_GBps"] = round(alg_total / (ms / 1000.0) / 1e9, 1)
        rec["algorithmic_frac"] = round(alg_total / (ms / 1000.0) / 1e9 / PEAK_HBM_GBS, 4)
    return rec


def roofline_of(rec, workload):
    """Roofline record of the dominant kernel family of a measured graph."""
    prof, stats = rec["_prof"], rec["_stats"]
    if not prof:
        return None
    dom = max(prof, key=lambda k: prof[k]["ms"])
    p = prof[dom]
    launch_ms = p["ms"] / p["launches"]
    own = p["bytes"] / p["launches"]
    alg = dominant_launch_bytes(dom, stats)
    per_launch = alg if alg is not None else own
    achieved = per_launch / (launch_ms / 1000.0) / 1e9
    traffic = load_traffic(dom, workload)
    r = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS,
         "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": traffic,
         "launch_ms": round(launch_ms, 4), "algorithmic_bytes_per_launch": per_launch,
         "bytes_model": "per-step algorithmic bytes" if alg is not None else
                        "kernel's own minimum bytes",
         "own_bytes_per_launch": own,
         "own_frac": round(own / (launch_ms / 1000.0) / 1e9 / PEAK_HBM_GBS, 4)}
    if traffic:
        tg = traffic / (launch_ms / 1000.0) / 1e9
        r["traffic_GBps"] = round(tg, 1)
        r["traffic_frac"] = round(tg / PEAK_HBM_GBS, 4)
    return r


def public(rec):
    return {k: v for k, v in rec.items() if not k.startswith("_")}


def to_device(u, v, w):
    import numpy as np
    import torch
    dev = torch.device("cuda:0")
    return [torch.from_numpy(np.ascontiguousarray(x).view(np.int32)).to(dev) for x in (u, v, w)]


def copy_bandwidth(dev, nbytes=1 << 31, reps=5):
    """Attainable HBM bandwidth: a plain device-to-device copy of nbytes, bytes
    read plus bytes written per second (GB/s)."""
    import torch
    a = torch.empty(nbytes, dtype=torch.uint8, device=dev).fill_(1)
    b = torch.empty_like(a)
    for _ in range(2):
        b.copy_(a)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    gbs = 2.0 * nbytes * reps / (time.perf_counter() - t) / 1e9
    del a, b
    torch.cuda.empty_cache()
    return gbs


# ------------------------------------------------------------- CPU baseline

def cpu_baseline(u, v, w, n, sample_edges, runs=3):
    """The oracle's Kruskal on the first `sample_edges` edges of the same
    graph (same n), single-threaded: one warm-up, then `runs` timed runs."""
    import oracle
    k = min(sample_edges, len(u))
    su, sv, sw = u[:k].copy(), v[:k].copy(), w[:k].copy()
    oracle.kruskal(su, sv, sw, n)
    times = []
    for _ in range(runs):
        t = time.perf_counter()
        oracle.kruskal(su, sv, sw, n)
        times.append(time.perf_counter() - t)
    mean = sum(times) / len(times)
    return {"value": k / mean, "unit": "edges/s", "cores": 1, "kind": "oracle",
            "sample": f"first {k} edges of the same graph (n={n}), single-threaded C "
                      f"Kruskal; 1 warm-up + {runs} timed runs, value from the mean",
            "seconds_mean": round(mean, 3), "seconds_min": round(min(times), 3),
            "value_best": k / min(times), "host_nproc": os.cpu_count()}


# ------------------------------------------------------------------ batch

def run_batch_workload(msf, graphs, steps, warmup, plain_sample, autotune):
    """The batch of GNM graphs (n log-uniform in [2^8, 2^18], average degree
    uniform in [4, 64], w uniform in [1, 2^31)): one hipGraph-captured
    persistent launch per step, against a loop of per-graph msf_compute calls
    on the first graphs of the batch."""
    import numpy as np
    import torch

    import graphgen

    G = graphs
    t = time.perf_counter()
    u, v, w, eo, vo = graphgen.batch_gnm(G, lo=8, hi=18, dlo=4, dhi=64, wlo=1, whi=2**31 - 1,
                                         seed=6)
    m = int(eo[-1])
    log(f"batch: generated {G} graphs, {m} edges in {time.perf_counter() - t:.1f}s")
    tu, tv, tw = to_device(u, v, w)
    b = msf.Batch(tu, tv, tw, eo, vo)
    torch.cuda.synchronize()
    tuned = b.autotune() if autotune else None
    if tuned:
        log(f"batch: autotuned {tuned}")
    b.capture()
    ms_batch, _ = timed(b.replay, steps, warmup)
    ticks = b.ticks.cpu().numpy().view(np.uint64).astype(np.float64)
    khz = msf.wall_clock_khz()
    fin, t0, start = ticks[:G], ticks[G], ticks[G + 1:]
    done_ms = (fin - t0) / khz
    serv_ms = (fin - start) / khz
    log(f"batch: {ms_batch:.2f} ms per batch, {G / ms_batch * 1000:.0f} graphs/s")

    k = min(plain_sample, G)
    max_e = int((eo[1:k + 1] - eo[:k]).max())
    max_n = int((vo[1:k + 1] - vo[:k]).max())
    ws = torch.empty(msf.workspace_bytes(max_e, max_n), dtype=torch.uint8, device=tu.device)
    mk = torch.empty(max(max_e, 1), dtype=torch.uint8, device=tu.device)
    for g in range(min(k, 20)):            # warm-up
        a, c = int(eo[g]), int(eo[g + 1])
        msf.compute(tu[a:c], tv[a:c], tw[a:c], int(vo[g + 1] - vo[g]), workspace=ws,
                    mask_out=mk[:c - a])
    torch.cuda.synchronize()
    per = []
    t0p = time.perf_counter()
    for g in range(k):
        a, c = int(eo[g]), int(eo[g + 1])
        tg = time.perf_counter()
        msf.compute(tu[a:c], tv[a:c], tw[a:c], int(vo[g + 1] - vo[g]), workspace=ws,
                    mask_out=mk[:c - a])
        per.append(time.perf_counter() - tg)
    torch.cuda.synchronize()
    plain_gps = k / (time.perf_counter() - t0p)
    batch_gps = G / (ms_batch / 1000.0)
    log(f"batch: plain {plain_gps:.0f} graphs/s over {k} graphs")

    # the oracle on the same sample, one core
    import oracle
    tc = time.perf_counter()
    for g in range(k):
        a, c = int(eo[g]), int(eo[g + 1])
        oracle.kruskal(u[a:c], v[a:c], w[a:c], int(vo[g + 1] - vo[g]))
    cpu_gps = k / (time.perf_counter() - tc)
    # the same graphs over all host cores (the oracle's C code runs without the GIL)
    from concurrent.futures import ThreadPoolExecutor
    threads = os.cpu_count() or 1

    def one(g):
        a, c = int(eo[g]), int(eo[g + 1])
        oracle.kruskal(u[a:c], v[a:c], w[a:c], int(vo[g + 1] - vo[g]))

    tc = time.perf_counter()
    with ThreadPoolExecutor(threads) as pool:
        list(pool.map(one, range(k)))
    cpu_par_gps = k / (time.perf_counter() - tc)
    del b, ws, mk, tu, tv, tw
    torch.cuda.empty_cache()
    return {
        "workload": BATCH_WORKLOAD, "graphs": G, "edges": m,
        "graphs_per_s": batch_gps, "ms_per_batch": round(ms_batch, 3), "steps": steps,
        "batched_edges_per_s": m / (ms_batch / 1000.0),
        "plain_graphs_per_s": plain_gps, "plain_sample": k,
        "speedup_vs_plain": batch_gps / plain_gps,
        "completion_ms": {"p50": float(np.percentile(done_ms, 50)),
                          "p99": float(np.percentile(done_ms, 99)),
                          "max": float(done_ms.max())},
        "service_ms": {"p50": float(np.percentile(serv_ms, 50)),
                       "p99": float(np.percentile(serv_ms, 99)),
                       "max": float(serv_ms.max())},
        "plain_service_ms": {"p50": 1000 * float(np.percentile(per, 50)),
                             "p99": 1000 * float(np.percentile(per, 99))},
        "cpu_oracle_graphs_per_s": cpu_gps,
        "cpu_oracle_parallel_graphs_per_s": cpu_par_gps, "cpu_oracle_threads": threads,
        "autotuned": tuned,
    }


# ------------------------------------------------------------------ extras

EXTRA_WORKLOADS = [("C1", "gnm_n2^16_m2^20"), ("C3a", "grid_4096x4096_keep0.8_w1e6"),
                   ("C3a_w255", "grid_4096x4096_keep0.8_w255"), ("C3b", "rgg2d_n2^24_deg8"),
                   ("rgg3d", "rgg3d_n2^24_deg16_w254"), ("rhg", "rhg_n2^24_deg16_g3_w254")]
FILTER_WORKLOAD = "rmat_n2^22_m2^28_w2^31"


def run_extras(msf, args):
    import torch

    import graphgen
    out = {}
    steps, warmup = max(1, min(args.steps, 10)), max(1, min(args.warmup, 3))
    for tag, name in EXTRA_WORKLOADS:
        t = time.perf_counter()
        u, v, w, n = graphgen.workload(name)
        log(f"{tag}: generated {name} in {time.perf_counter() - t:.1f}s")
        tu, tv, tw = to_device(u, v, w)
        rec = measure_graph(msf, tu, tv, tw, n, name, steps, warmup, 2)
        rec["roofline"] = roofline_of(rec, name)
        out[tag] = public(rec)
        log(f"{tag}: {rec['ms_per_step']:.3f} ms/step, {rec['edges_per_s']:.3e} edges/s")
        del tu, tv, tw
        torch.cuda.empty_cache()

    # C4: Filter-Borůvka, the pivot network against the sampled median and
    # against plain Borůvka on the same graph
    t = time.perf_counter()
    u, v, w, n = graphgen.workload(FILTER_WORKLOAD)
    log(f"C4: generated {FILTER_WORKLOAD} in {time.perf_counter() - t:.1f}s")
    tu, tv, tw = to_device(u, v, w)
    msf.load_pivot_model()
    try:
        net = measure_graph(msf, tu, tv, tw, n, FILTER_WORKLOAD, steps, warmup, 2,
                            algo="filter", pivot="mlp")
    finally:
        msf.clear_pivot_model()
    med = measure_graph(msf, tu, tv, tw, n, FILTER_WORKLOAD, steps, warmup, 1,
                        algo="filter", pivot="median")
    plain = measure_graph(msf, tu, tv, tw, n, FILTER_WORKLOAD, steps, warmup, 1)
    if not (net["total_weight"] == med["total_weight"] == plain["total_weight"]):
        raise RuntimeError("C4: the three solvers gave different totals")
    q = net["_stats"]["pivot_q_used"]
    net["roofline"] = roofline_of(net, FILTER_WORKLOAD)
    out["C4"] = {"network": public(net), "network_q": q,
                 "median_ms_per_step": med["ms_per_step"],
                 "plain_boruvka_ms_per_step": plain["ms_per_step"],
                 "speedup_vs_median": round(med["ms_per_step"] / net["ms_per_step"], 4),
                 "speedup_vs_plain": round(plain["ms_per_step"] / net["ms_per_step"], 4)}
    log(f"C4: network {net['ms_per_step']:.3f} ms (q={q:.3f}), median "
        f"{med['ms_per_step']:.3f} ms, plain {plain['ms_per_step']:.3f} ms")
    del tu, tv, tw
    torch.cuda.empty_cache()

    if args.graphs > 0:
        out["C5"] = run_batch_workload(msf, args.graphs, max(1, min(args.steps, 3)), 1,
                                       args.plain_sample, args.autotune)
    return out


# -------------------------------------------------------------------- main

def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD)
    ap.add_argument("--algo", default="boruvka", choices=["boruvka", "filter"])
    ap.add_argument("--pivot", default="median")
    ap.add_argument("--quantile", type=float, default=0.5)
    ap.add_argument("--model", default=None, help="pivot network file (--pivot mlp)")
    ap.add_argument("--no-extras", action="store_true",
                    help="measure only the named workload (no other configurations)")
    ap.add_argument("--cpu-sample", type=int, default=1 << 26,
                    help="edges given to the timed CPU oracle (0 = skip)")
    ap.add_argument("--graphs", type=int, default=10000, help="batch workload: graphs (0 = skip)")
    ap.add_argument("--plain-sample", type=int, default=300,
                    help="batch workload: graphs timed with per-graph calls")
    ap.add_argument("--autotune", action=argparse.BooleanOptionalAction, default=True,
                    help="batch workload: autotune the batched launch first")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (calibrates byte counters)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: this library runs on one GPU; multi-GPU runs are not part of it "
              f"(asked for --gpus {args.gpus}, WORLD_SIZE={world}).", file=sys.stderr)
        sys.exit(2)

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

    import paper_2302_12199_amd as msf

    if args.workload == BATCH_WORKLOAD:
        rec = run_batch_workload(msf, args.graphs, args.steps, args.warmup, args.plain_sample,
                                 args.autotune)
        out = {"metric": "batched graphs/s (10,000 GNM graphs) vs per-graph plain calls",
               "value": rec["graphs_per_s"], "unit": "graphs/s", "n_gpus": 1,
               "steps": args.steps, "warmup": args.warmup, "ms_per_step": rec["ms_per_batch"],
               "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
               "dtype": "u64", "data": "synthetic",
               "config": {"workload": BATCH_WORKLOAD, "graphs": rec["graphs"],
                          "edges": rec["edges"]}, "batch": rec}
        print(json.dumps(out), flush=True)
        return

    import graphgen

    t = time.perf_counter()
    u, v, w, n = graphgen.workload(args.workload)
    m = len(u)
    log(f"generated {args.workload}: n={n} m={m} in {time.perf_counter() - t:.1f}s")
    tu, tv, tw = to_device(u, v, w)
    opts = dict(algo=args.algo, pivot=args.pivot, quantile=args.quantile)
    if args.algo == "filter" and args.pivot == "mlp":
        msf.load_pivot_model(args.model)        # default: the shipped network
    import torch
    log(f"resident on {torch.cuda.get_device_name(tu.device)}")
    rec = measure_graph(msf, tu, tv, tw, n, args.workload, args.steps, args.warmup, 2, **opts)
    log(f"timed {args.steps} steps: {rec['ms_per_step']:.3f} ms/step total={rec['total_weight']}")
    roofline = roofline_of(rec, args.workload)
    dev = tu.device
    del tu, tv, tw
    torch.cuda.empty_cache()
    if roofline:
        cg = copy_bandwidth(dev)
        roofline["copy_GBps"] = round(cg, 1)
        roofline["achieved_vs_copy"] = round(roofline["achieved"] / cg, 4)
        log(f"attainable copy bandwidth {cg:.0f} GB/s")

    cpu = None
    if args.cpu_sample > 0:
        cpu = cpu_baseline(u, v, w, n, args.cpu_sample)
        log(f"cpu oracle: {cpu['value']:.3e} edges/s ({cpu['sample']})")
    del u, v, w

    extras = None
    if not args.no_extras and args.workload == DEFAULT_WORKLOAD and args.algo == "boruvka":
        extras = run_extras(msf, args)

    stats = rec["_stats"]
    out = {
        "metric": METRIC, "value": rec["edges_per_s"], "unit": "edges/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": rec["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": args.workload, "n": int(n), "m": int(m), "algo": args.algo,
                   "pivot": args.pivot if args.algo == "filter" else None},
        "roofline": roofline, "cpu_baseline": cpu,
        "algorithmic_GBps": rec.get("algorithmic_GBps"),
        "algorithmic_frac": rec.get("algorithmic_frac"),
        "pivot_vs_median": extras["C4"] if extras else None,
        "batched": extras.get("C5") if extras else None,
        "configs": {k: x for k, x in extras.items() if k not in ("C4", "C5")} if extras else None,
        "detail": {"rounds": stats["rounds"], "round_live": stats["round_live"],
                   "round_edges": stats["round_edges"],
                   "round_vertices": stats["round_vertices"], "msf_edges": stats["msf_edges"],
                   "total_weight": stats["total_weight"], "kernels": rec["kernels"],
                   "timing": "timed steps with the kernel profiler off; kernel table from "
                             "2 separate profiled steps"},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
