#!/usr/bin/env python3
"""Benchmark of the k-hop neighborhood count on one MI355X.

Workload (the paper's benchmark protocol of Section III on a synthetic stand-in
for its Graph500 dataset): R-MAT scale 21, edge factor 32, a/b/c/d =
0.57/0.19/0.19/0.05, symmetrised, self-loops and duplicates dropped; 300 seeds
at k = 1 and at k = 2, 10 seeds at k = 3 and at k = 6.

One step answers that query set twice, with the graph and the seeds already
resident in device memory:
  plain    one launch sequence per query, queries one after another;
  batched  all queries in seed-bitset launches (mixed k).
value = traversed edges credited to every answered query / step time (GTEPS),
where a query's credit is the out-degree sum of the vertices at distance
0..k-1 (the edges a top-down search inspects).

After the timed steps, the same steps run once more with per-kernel HIP-event
profiling for the roofline figure, per-query latencies are taken through the
host entry point, and (N = 1 only) the CPU oracle answers the query set on the
host for the baseline; its counts are also compared with the GPU's.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GTEPS and k-hop queries/sec (batched vs plain) on 1 MI355X; p50/p99 latency"
HBM_PEAK_GBS = 8000.0
PROTOCOL = ((1, 300, 0), (2, 300, 0), (3, 10, 1), (6, 10, 1))  # (k, seeds, seed stream)


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def build_queries(el):
    import graphgen
    groups = []
    draws = {}
    for k, count, stream in PROTOCOL:
        if stream not in draws:
            draws[stream] = graphgen.draw_seeds(el, 300 if stream == 0 else 10, seed=7, stream=stream)
        groups.append((k, draws[stream][:count].copy()))
    return groups


def pct(a, q):
    return float(np.percentile(np.asarray(a, dtype=np.float64), q)) if len(a) else None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--scale", type=int, default=21)
    ap.add_argument("--edge-factor", type=int, default=32)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-latency", action="store_true")
    ap.add_argument("--no-profile", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU design is "
              "described but not built", file=sys.stderr)
        sys.exit(2)

    import torch

    import graphgen
    import paper_1905_01294_amd as K

    t0 = time.time()
    el = graphgen.rmat(args.scale, args.edge_factor, seed=1)
    groups = build_queries(el)
    log(f"generated {el.m} tuples in {time.time() - t0:.1f}s")
    t0 = time.time()
    g = K.Graph.from_edgelist(el)
    log(f"device graph: n={g.n} arcs={g.num_arcs} in {time.time() - t0:.1f}s")

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    d_groups = []
    for k, seeds in groups:
        n = len(seeds)
        d_groups.append((k, torch.from_numpy(seeds).to(dev), torch.empty(n, dtype=torch.int64, device=dev),
                         torch.empty(n, dtype=torch.int64, device=dev)))
    all_seeds = np.concatenate([s for _, s in groups]).astype(np.int32)
    all_ks = np.concatenate([np.full(len(s), k, np.int32) for k, s in groups])
    d_all_seeds = torch.from_numpy(all_seeds).to(dev)
    d_all_ks = torch.from_numpy(all_ks).to(dev)
    d_batched = torch.empty(len(all_seeds), dtype=torch.int64, device=dev)
    nq = len(all_seeds)

    def plain_pass():
        for k, ds, dc, dt in d_groups:
            g.count_dev(ds, k, dc, dt, stream=stream)

    def batched_pass():
        g.count_batched_dev(d_all_seeds, d_all_ks, d_batched, stream=stream)

    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]

    def step(times=None):
        ev[0].record(stream)
        plain_pass()
        ev[1].record(stream)
        batched_pass()
        ev[2].record(stream)
        if times is not None:
            times.append(ev)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    plain_counts = torch.cat([dc for _, _, dc, _ in d_groups]).cpu().numpy()
    plain_te = torch.cat([dt for _, _, _, dt in d_groups]).cpu().numpy()
    batched_counts = d_batched.cpu().numpy()
    if not np.array_equal(plain_counts, batched_counts):
        raise SystemExit("batched counts differ from plain counts")
    te_set = int(plain_te.sum())

    # ---- timed region
    plain_ms, batched_ms = [], []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        step()
        ev[2].synchronize()
        plain_ms.append(ev[0].elapsed_time(ev[1]))
        batched_ms.append(ev[1].elapsed_time(ev[2]))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    ms_per_step = wall * 1000.0 / args.steps
    value = 2.0 * te_set / (wall / args.steps) / 1e9
    log(f"timed {args.steps} steps: {ms_per_step:.2f} ms/step, {value:.2f} GTEPS")
    p_ms = float(np.mean(plain_ms))
    b_ms = float(np.mean(batched_ms))

    # ---- profiled replay for the per-kernel roofline
    roofline = None
    kernels = None
    if not args.no_profile:
        g.profile(True)
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        kernels = g.profile_read()
        g.profile(False)
        dom_name, dom = max(kernels.items(), key=lambda kv: kv[1]["total_ms"])
        achieved = dom["algorithmic_bytes"] / (dom["total_ms"] / 1000.0) / 1e9 if dom["total_ms"] > 0 else 0.0
        roofline = {"kernel": dom_name, "bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                    "launches": dom["launches"], "avg_launch_us": round(1000.0 * dom["total_ms"] / dom["launches"], 3),
                    "algorithmic_bytes_per_launch": round(dom["algorithmic_bytes"] / dom["launches"], 1)}
        for name, kv in kernels.items():
            kv["gbs"] = round(kv["algorithmic_bytes"] / (kv["total_ms"] / 1000.0) / 1e9, 2) if kv["total_ms"] else 0
            kv["avg_us"] = round(1000.0 * kv["total_ms"] / max(kv["launches"], 1), 3)

    # ---- per-query latency through the host entry point (PCIe round trip included)
    latency = None
    if not args.no_latency:
        latency = {}
        for k, seeds in groups:
            lat = []
            for s in seeds:
                t = time.perf_counter()
                g.count(np.array([s], np.int32), k)
                lat.append((time.perf_counter() - t) * 1000.0)
            latency[f"k{k}"] = {"mean_ms": round(float(np.mean(lat)), 4), "p50_ms": round(pct(lat, 50), 4),
                                "p99_ms": round(pct(lat, 99), 4), "n": len(lat)}

    # ---- CPU oracle baseline (host cores, same queries)
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        t0 = time.time()
        og = oracle.OracleGraph.from_edgelist(el)
        log(f"oracle adjacency in {time.time() - t0:.1f}s")
        o_counts, o_te, o_lat = [], [], {}
        t_all = 0.0
        for k, seeds in groups:
            lat = []
            for s in seeds:
                t = time.perf_counter()
                c, te, _ = og.khop(int(s), k)
                dt = time.perf_counter() - t
                lat.append(dt * 1000.0)
                t_all += dt
                o_counts.append(c)
                o_te.append(te)
            o_lat[f"k{k}"] = {"mean_ms": round(float(np.mean(lat)), 3), "p50_ms": round(pct(lat, 50), 3),
                              "p99_ms": round(pct(lat, 99), 3)}
        parity = bool(np.array_equal(np.array(o_counts), plain_counts) and np.array_equal(np.array(o_te), plain_te))
        cpu = {"value": round(sum(o_te) / t_all / 1e9, 4), "unit": "GTEPS", "cores": 1, "kind": "oracle",
               "sample": f"the full query set once ({nq} queries: 300 at k=1, 300 at k=2, 10 at k=3, 10 at k=6), "
                         f"one query at a time on one host core; adjacency build excluded",
               "seconds": round(t_all, 2), "qps": round(nq / t_all, 2), "latency": o_lat,
               "counts_equal_gpu": parity, "host_cpu": _cpu_model(), "host_nproc": os.cpu_count()}
        if not parity:
            log("WARNING: oracle counts differ from the GPU counts")

    out = {
        "metric": METRIC, "value": round(value, 3), "unit": "GTEPS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": f"rmat{args.scale}_ef{args.edge_factor}_khop_protocol",
                   "graph": f"R-MAT scale {args.scale}, edge factor {args.edge_factor}, a/b/c/d 0.57/0.19/0.19/0.05, "
                            "undirected, self-loops and duplicates dropped",
                   "vertices": g.n, "arcs": g.num_arcs, "queries_per_pass": nq,
                   "k_mix": {"1": 300, "2": 300, "3": 10, "6": 10}, "passes_per_step": ["plain", "batched"],
                   "traversed_edges_per_pass": te_set},
        "plain": {"gteps": round(te_set / (p_ms / 1000.0) / 1e9, 3), "qps": round(nq / (p_ms / 1000.0), 1),
                  "ms_per_pass": round(p_ms, 3)},
        "batched": {"gteps": round(te_set / (b_ms / 1000.0) / 1e9, 3), "qps": round(nq / (b_ms / 1000.0), 1),
                    "ms_per_pass": round(b_ms, 3), "seeds_per_launch": g.get_option(K.KHOP_OPT_BATCH_SEEDS)},
        "batched_vs_plain_qps": round(p_ms / b_ms, 3),
        "latency_host_api": latency,
        "roofline": roofline,
        "kernels": kernels,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    g.free()


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


if __name__ == "__main__":
    main()
