#!/usr/bin/env python3
"""Benchmark of the k-hop neighborhood count on one MI355X.

Workload (the paper's benchmark protocol of Section III on a synthetic stand-in
for its Graph500 dataset): R-MAT scale 21, edge factor 32, a/b/c/d =
0.57/0.19/0.19/0.05, symmetrised, self-loops and duplicates dropped; 300 seeds
at k = 1 and at k = 2, 10 seeds at k = 3 and at k = 6.

One step answers that query set twice, with the graph and the seeds already
resident in device memory:
  plain    the plain single-query path in one device call per k: queries are
           answered in order, and consecutive queries overlap by one launch
           (the last hop of one beside hop 1 of the next);
  batched  all queries in seed-bitset launches (mixed k).
value = traversed edges credited to every answered query / step time (GTEPS),
where a query's credit is the out-degree sum of the vertices at distance
0..k-1 (the edges a top-down search inspects).

Beside the step: the strictly sequential plain form (one launch sequence per
query, each complete before the next starts), the 32-seed scale-10 case, the
autotuner's search (live, unless a cache is named), per-kernel HIP-event
profiling for the roofline figure, per-query latencies through the host entry
point, the batched seeds-per-launch sweep, full-depth search, neighborhood
sets and label-filtered counts, the 41.6M-vertex power-law graph (its plain
protocol and a 256-seed batch), serving (the scale-21 graph alone, then both
graphs resident), and (N = 1 only) the CPU oracle answering the query set on
the host for the baseline, its counts compared with the GPU's.
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
    ap.add_argument("--no-sweep", action="store_true", help="skip the batched seeds-per-launch sweep")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving measurement")
    ap.add_argument("--no-bfs", action="store_true",
                    help="skip the breadth-first search, neighborhood-set and level measurements")
    ap.add_argument("--only-bfs", action="store_true",
                    help="print only the breadth-first search, neighborhood-set and level measurements (one JSON "
                         "line, not the benchmark line)")
    ap.add_argument("--step-only", action="store_true",
                    help="run only the timed steps and their profiled replay (for profiling the step with rocprofv3)")
    ap.add_argument("--only-serving", action="store_true",
                    help="print only the serving measurements (one JSON line, not the benchmark line)")
    ap.add_argument("--no-twitter", action="store_true",
                    help="skip the 41.6M-vertex power-law graph (its legs and two-graph serving)")
    ap.add_argument("--tune-cache", default=None,
                    help="autotuner cache file to read and write (default: a fresh one, so the search runs)")
    ap.add_argument("--serve-seconds", type=float, default=2.0, help="arrival window per offered-load level")
    ap.add_argument("--no-autotune", action="store_true", help="time the default settings instead of tuned ones")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy 256 MiB device buffers (the known-size kernel that scales PMC byte counters)")
    ap.add_argument("--pmc-summary", metavar="DIR",
                    help="summarise rocprofv3 --pmc FETCH_SIZE/WRITE_SIZE CSVs (bench_* and copy_*) in DIR as JSON")
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.pmc_summary:
        print(json.dumps(pmc_summary(args.pmc_summary), indent=1))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU design is "
              "described but not built", file=sys.stderr)
        sys.exit(2)

    # the autotuner's cache: a fresh file unless one is named, so the settings are searched for the
    # kernels being timed (the cache key also carries a hash of the library's sources)
    import tempfile
    tune_dir = None
    if args.tune_cache:
        os.environ["KHOP_TUNE_CACHE"] = args.tune_cache
    else:
        tune_dir = tempfile.mkdtemp(prefix="khop_tune_")
        os.environ["KHOP_TUNE_CACHE"] = os.path.join(tune_dir, "tune.txt")
    legs = {}
    t_bench = time.time()
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
    tuning = {"rmat21": run_autotune(g, K, "rmat21")} if not args.no_autotune else None
    legs["load_and_tune_s"] = round(time.time() - t_bench, 2)

    if args.only_serving:
        out = {"rmat21": serving_bench(K, [("rmat21", g, el)], args.serve_seconds)}
        if not args.no_twitter:
            el2 = graphgen.twitter_like(seed=1)
            g2 = K.Graph.from_edgelist(el2)
            if not args.no_autotune:
                run_autotune(g2, K, "chunglu41.6M")
            out["rmat21+chunglu41.6M"] = serving_bench(K, [("rmat21", g, el), ("chunglu41.6M", g2, el2)],
                                                       args.serve_seconds)
            g2.free()
        print(json.dumps(out), flush=True)
        g.free()
        return

    if args.only_bfs:
        cpu_leg = not args.no_cpu_baseline
        print(json.dumps({"bfs": bfs_bench(g, el, K, torch, cpu_leg=cpu_leg),
                          "neighborhood_sets": sets_bench(g, el, groups, K, torch, cpu_leg=cpu_leg),
                          "label_filtered": filtered_bench(g, el, groups, K, torch, cpu_leg=cpu_leg)}), flush=True)
        g.free()
        return

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
    legs["step_s"] = round(time.time() - t_bench - legs["load_and_tune_s"], 2)

    if args.step_only:
        for flag in ("no_cpu_baseline", "no_latency", "no_sweep", "no_serving", "no_bfs", "no_twitter"):
            setattr(args, flag, True)
    # ---- the strictly sequential plain form: one launch sequence per query, each complete (count
    # written) before the next query's first launch, on the same device-resident queries
    t_leg = time.time()
    s_ms, g0_leg = float("nan"), None
    if not args.step_only:
        g.set_option(K.KHOP_OPT_PLAIN_PIPELINE, 0)
        plain_pass()
        plain_pass()
        torch.cuda.synchronize()
        seq_counts = torch.cat([dc for _, _, dc, _ in d_groups]).cpu().numpy()
        ev[0].record(stream)
        for _ in range(3):
            plain_pass()
        ev[1].record(stream)
        ev[1].synchronize()
        g.set_option(K.KHOP_OPT_PLAIN_PIPELINE, 1)
        s_ms = ev[0].elapsed_time(ev[1]) / 3
        if not np.array_equal(seq_counts, plain_counts):
            raise SystemExit("sequential plain counts differ from the pipelined ones")
        log(f"sequential plain pass: {s_ms:.3f} ms ({nq / (s_ms / 1e3):.0f} queries/s)")
        g0_leg = g0_bench(K, torch, cpu_leg=not args.no_cpu_baseline)
    legs["sequential_and_g0_s"] = round(time.time() - t_leg, 2)

    # ---- profiled replay for the per-kernel roofline
    roofline = None
    kernels = None
    if not args.no_profile:
        g.profile(True)
        for _ in range(min(args.steps, 3)):
            step()
        torch.cuda.synchronize()
        kernels = g.profile_read()
        g.profile(False)
        # the event bracket's own time, from empty launches timed the same way
        empty = kernels.pop("empty_launch", None)
        overhead_us = 1000.0 * empty["total_ms"] / empty["launches"] if empty and empty["launches"] else 0.0
        for name, kv in kernels.items():
            kv["event_avg_us"] = round(1000.0 * kv["total_ms"] / max(kv["launches"], 1), 3)
            kv["avg_us"] = round(max(kv["event_avg_us"] - overhead_us, 0.0), 3)
            kv["gbs"] = round(kv["algorithmic_bytes"] / kv["launches"] / (kv["avg_us"] * 1e-6) / 1e9, 2) \
                if kv["avg_us"] > 0 else 0
        dom_name, dom = max(kernels.items(), key=lambda kv: kv[1]["launches"] * kv[1]["avg_us"])
        achieved = dom["gbs"]
        tr = traffic_per_launch(dom_name)
        copy_gbs = measure_copy_gbs(torch)
        # time-weighted aggregate over the traversal kernels
        trav_kinds = ("plain_step", "plain_hop_push", "plain_hop_pull", "plain_compact", "batch_pull",
                      "batch_pull_heavy")
        trav = [kv for name, kv in kernels.items() if name in trav_kinds]
        trav_s = sum(kv["avg_us"] * kv["launches"] for kv in trav) * 1e-6
        trav_gbs = sum(kv["algorithmic_bytes"] for kv in trav) / trav_s / 1e9 if trav_s > 0 else 0.0
        roofline = {"kernel": dom_name, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                    "traffic": round(tr, 1) if tr is not None else None, "traffic_unit": "bytes per launch",
                    "launches": dom["launches"], "avg_launch_us": dom["avg_us"],
                    "event_avg_launch_us": dom["event_avg_us"], "event_overhead_us": round(overhead_us, 3),
                    "algorithmic_bytes_per_launch": round(dom["algorithmic_bytes"] / dom["launches"], 1),
                    "copy_ceiling_gbs": round(copy_gbs, 1), "frac_of_copy": round(achieved / copy_gbs, 4),
                    "traversal_aggregate": {"kernels": list(trav_kinds),
                                            "achieved": round(trav_gbs, 1),
                                            "frac": round(trav_gbs / HBM_PEAK_GBS, 4),
                                            "frac_of_copy": round(trav_gbs / copy_gbs, 4)},
                    # the plain path's hops 2..k-1 (the levels that carry its bytes) and the batched
                    # bottom-up kernels, each against the peak
                    "by_role": {name: {"achieved": kernels[name]["gbs"],
                                       "frac": round(kernels[name]["gbs"] / HBM_PEAK_GBS, 4),
                                       "avg_launch_us": kernels[name]["avg_us"],
                                       "launches": kernels[name]["launches"]}
                                for name in ("plain_step", "plain_hop_push", "plain_hop_pull", "plain_compact",
                                             "batch_pull", "batch_pull_heavy") if name in kernels}}

    # ---- per-query latency through the host entry point (PCIe round trip included)
    latency = None
    if not args.no_latency:
        latency = {}
        # Python's cyclic garbage collector, not the library, can pause a call for tens of milliseconds
        # in a process this size: it is run first and kept off while calls are timed
        import gc
        gc.collect()
        gc.disable()
        for k, seeds in groups:
            lat = []
            for s in seeds:
                t = time.perf_counter()
                g.count(np.array([s], np.int32), k)
                lat.append((time.perf_counter() - t) * 1000.0)
            worst = int(np.argmax(lat))
            latency[f"k{k}"] = {"mean_ms": round(float(np.mean(lat)), 4), "p50_ms": round(pct(lat, 50), 4),
                                "p99_ms": round(pct(lat, 99), 4), "max_ms": round(float(np.max(lat)), 4),
                                "max_at": {"index": worst, "seed": int(seeds[worst])}, "n": len(lat)}
        gc.enable()

    t_leg = time.time()
    sweep = None if args.no_sweep else batched_sweep(g, el, K, torch)
    bfs = None if args.no_bfs else bfs_bench(g, el, K, torch, cpu_leg=not args.no_cpu_baseline)
    sets = None if args.no_bfs else sets_bench(g, el, groups, K, torch, cpu_leg=not args.no_cpu_baseline)
    filtered = None if args.no_bfs else filtered_bench(g, el, groups, K, torch, cpu_leg=not args.no_cpu_baseline)
    legs["sweep_bfs_sets_filtered_s"] = round(time.time() - t_leg, 2)
    g2 = el2 = None
    power_law = None
    if not args.no_twitter:
        t_leg = time.time()
        el2 = graphgen.twitter_like(seed=1)
        g2 = K.Graph.from_edgelist(el2)
        log(f"power-law graph: n={g2.n} arcs={g2.num_arcs} in {time.time() - t_leg:.1f}s")
        legs["power_law_load_s"] = round(time.time() - t_leg, 2)
        t_leg = time.time()
        if not args.no_autotune:
            tuning["chunglu41.6M"] = run_autotune(g2, K, "chunglu41.6M")
        power_law = power_law_bench(g2, el2, K, torch)
        legs["power_law_s"] = round(time.time() - t_leg, 2)
    serving = None
    if not args.no_serving:
        t_leg = time.time()
        serving = {"rmat21": serving_bench(K, [("rmat21", g, el)], args.serve_seconds)}
        if g2 is not None:
            serving["rmat21+chunglu41.6M"] = serving_bench(K, [("rmat21", g, el), ("chunglu41.6M", g2, el2)],
                                                           args.serve_seconds)
        legs["serving_s"] = round(time.time() - t_leg, 2)
    if g2 is not None:
        g2.free()

    # ---- CPU oracle baseline (host cores, same queries)
    cpu = None
    t_leg = time.time()
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
        # the same queries over a pool of host threads, one query per thread at a time
        from concurrent.futures import ThreadPoolExecutor
        threads = min(os.cpu_count() or 1, 16)
        jobs = [(int(s), k) for k, seeds in groups for s in seeds]
        t = time.perf_counter()
        with ThreadPoolExecutor(threads) as ex:
            pool_counts = list(ex.map(lambda j: og.khop(j[0], j[1])[0], jobs))
        pool_s = time.perf_counter() - t
        parity = parity and bool(np.array_equal(np.array(pool_counts), plain_counts))
        cpu = {"value": round(sum(o_te) / t_all / 1e9, 4), "unit": "GTEPS", "cores": 1, "kind": "oracle",
               "sample": f"the full query set once ({nq} queries: 300 at k=1, 300 at k=2, 10 at k=3, 10 at k=6), "
                         f"one query at a time on one host core; adjacency build excluded",
               "seconds": round(t_all, 2), "qps": round(nq / t_all, 2), "latency": o_lat,
               "counts_equal_gpu": parity, "host_cpu": _cpu_model(), "host_nproc": os.cpu_count(),
               "pool": {"threads": threads, "seconds": round(pool_s, 3), "qps": round(nq / pool_s, 1),
                        "gteps": round(sum(o_te) / pool_s / 1e9, 4)}}
        if not parity:
            log("WARNING: oracle counts differ from the GPU counts")
    legs["cpu_baseline_s"] = round(time.time() - t_leg, 2)
    legs["total_s"] = round(time.time() - t_bench, 2)
    if tune_dir:
        import shutil
        shutil.rmtree(tune_dir, ignore_errors=True)

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
        "plain": {"form": "pipelined: queries in order, consecutive queries overlap by one launch",
                  "gteps": round(te_set / (p_ms / 1000.0) / 1e9, 3), "qps": round(nq / (p_ms / 1000.0), 1),
                  "ms_per_pass": round(p_ms, 3)},
        "plain_sequential": None if args.step_only else {
            "form": "one launch sequence per query, each complete before the next starts",
            "gteps": round(te_set / (s_ms / 1000.0) / 1e9, 3), "qps": round(nq / (s_ms / 1000.0), 1),
            "ms_per_pass": round(s_ms, 3)},
        "batched": {"gteps": round(te_set / (b_ms / 1000.0) / 1e9, 3), "qps": round(nq / (b_ms / 1000.0), 1),
                    "ms_per_pass": round(b_ms, 3), "seeds_per_launch": g.get_option(K.KHOP_OPT_BATCH_SEEDS)},
        "batched_vs_plain_qps": round(p_ms / b_ms, 3),
        "batched_vs_plain_sequential_qps": None if args.step_only else round(s_ms / b_ms, 3),
        "g0_plain": g0_leg,
        "tuning": tuning,
        "legs_seconds": legs,
        "latency_host_api": latency,
        "batched_sweep": sweep,
        "serving": serving,
        "bfs": bfs,
        "neighborhood_sets": sets,
        "label_filtered": filtered,
        "roofline": roofline,
        "kernels": kernels,
        "cpu_baseline": cpu,
        "device": device_info(torch),
        "power_law": power_law,
    }
    print(json.dumps(out), flush=True)
    g.free()


TUNED_OPTIONS = (("alpha", "KHOP_OPT_ALPHA"), ("beta", "KHOP_OPT_BETA"), ("pull_light", "KHOP_OPT_PULL_LIGHT"),
                 ("pull_heavy", "KHOP_OPT_PULL_HEAVY"), ("push_atomic", "KHOP_OPT_PUSH_ATOMIC"),
                 ("plain_grid", "KHOP_OPT_PLAIN_GRID"), ("batch_seeds", "KHOP_OPT_BATCH_SEEDS"),
                 ("batch_heavy", "KHOP_OPT_BATCH_HEAVY"), ("batch_push_div", "KHOP_OPT_BATCH_PUSH"),
                 ("batch_grid", "KHOP_OPT_BATCH_GRID"))


def run_autotune(g, K, name):
    """khop_autotune on a graph: whether it searched or read the cache, how long it took, what it chose."""
    t0 = time.time()
    g.autotune(0)
    secs = time.time() - t0
    searched = K.khop_autotune_seconds()
    settings = {key: g.get_option(getattr(K, opt)) for key, opt in TUNED_OPTIONS}
    log(f"{name}: autotune {'searched' if searched > 0 else 'read from the cache'} in {secs:.1f}s: {settings}")
    return {"source": "search" if searched > 0 else "cache", "seconds": round(secs, 2), "settings": settings,
            "library": K.khop_version()}


def g0_bench(K, torch, cpu_leg=True):
    """The 32-seed scale-10 case (R-MAT scale 10, edge factor 16) through the plain path at k = 1, 2, 3, 6."""
    import graphgen
    el0 = graphgen.rmat(10, 16, seed=1)
    seeds = graphgen.draw_seeds(el0, 32, seed=7)
    g0 = K.Graph.from_edgelist(el0)
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    d_s = torch.from_numpy(seeds).to(dev)
    out = {"graph": "R-MAT scale 10, edge factor 16", "seeds": 32}
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    counts = {}
    for k in (1, 2, 3, 6):
        d_c = torch.empty(32, dtype=torch.int64, device=dev)
        for _ in range(2):  # (a repeated run replays the launches captured when it is seen again)
            g0.count_dev(d_s, k, d_c, stream=stream)
        e0.record(stream)
        for _ in range(10):
            g0.count_dev(d_s, k, d_c, stream=stream)
        e1.record(stream)
        e1.synchronize()
        ms = e0.elapsed_time(e1) / 10
        counts[k] = d_c.cpu().numpy()
        out[f"k{k}"] = {"ms": round(ms, 4), "qps": round(32 / (ms / 1e3), 1)}
    if cpu_leg:
        import oracle
        og = oracle.OracleGraph.from_edgelist(el0)
        out["equal_oracle"] = all(bool(np.array_equal(counts[k], og.count(seeds, k)[0])) for k in counts)
    g0.free()
    log(f"scale-10 plain: {out}")
    return out


KERNEL_SOURCES = {"plain": "paper_1905_01294_amd/csrc/plain.hip", "batch": "paper_1905_01294_amd/csrc/batched.hip"}


def _source_sha(kernel):
    import hashlib
    path = os.path.join(ROOT, KERNEL_SOURCES[kernel.split("_")[0]])
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


# GPU kernel name stem -> the kernel kind khop_profile reports it under
KERNEL_KIND = {"plain_close": "plain_init", "plain_final": "plain_init", "plain_step": "plain_step",
               "batch_zero": "batch_init", "batch_narrow": "batch_init", "batch_push_seeds": "batch_push",
               "batch_row_count": "batch_push", "batch_seed": "batch_init", "batch_frontier_copy": "batch_init",
               "batch_output": "batch_count"}


def pmc_summary(d, copy_bytes=256 << 20):
    """Mean FETCH_SIZE / WRITE_SIZE (KiB per dispatch) per library kernel, with the
    factors that make the counters read a 256 MiB copy as 256 MiB each way."""
    import csv
    import re
    out = {"fetch_scale": None, "write_scale": None, "kernels": {}}
    for c, key in (("FETCH_SIZE", "fetch"), ("WRITE_SIZE", "write")):
        rows = csv.DictReader(open(os.path.join(d, f"copy_{c}_counter_collection.csv")))
        vals = [float(r["Counter_Value"]) for r in rows
                if "copyBuffer" in r["Kernel_Name"]]
        out[f"{key}_scale"] = round(copy_bytes / 1024.0 / (sum(vals) / len(vals)), 4)
        acc = {}
        for r in csv.DictReader(open(os.path.join(d, f"bench_{c}_counter_collection.csv"))):
            m = re.search(r"(plain_[a-z]+|batch_[a-z_]+?)\d*_kernel", r["Kernel_Name"])
            if m:
                kind = KERNEL_KIND.get(m.group(1), m.group(1))
                acc.setdefault(kind, []).append(float(r["Counter_Value"]))
        for k, v in acc.items():
            e = out["kernels"].setdefault(k, {"source_sha256_16": _source_sha(k)})
            e[f"{key}_kib_per_dispatch"] = round(sum(v) / len(v), 1)
            e["dispatches"] = len(v)
    return out


def traffic_per_launch(kernel):
    """HBM bytes per launch of `kernel` from the step kernels PMC summary under profiles/, or None when absent or
    when the kernel's source changed after the counters were taken."""
    import re
    path = os.path.join(ROOT, "profiles", "step_kernels_rmat21_pmc_traffic.md")
    if not os.path.exists(path):
        return None
    m = re.search(r"```json\n(.*?)```", open(path).read(), re.S)
    if not m:
        return None
    d = json.loads(m.group(1))
    e = d["kernels"].get(kernel)
    if not e or e.get("source_sha256_16") != _source_sha(kernel):
        return None
    return 1024.0 * (e["fetch_kib_per_dispatch"] * d["fetch_scale"] + e["write_kib_per_dispatch"] * d["write_scale"])


def measure_copy_gbs(torch, nbytes=1 << 30, reps=10):
    """Device-to-device copy rate (bytes read + written per second): the practical streaming ceiling."""
    a = torch.ones(nbytes // 4, dtype=torch.int32, device="cuda:0")
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    gbs = 2.0 * nbytes * reps / (e0.elapsed_time(e1) / 1000.0) / 1e9
    del a, b
    return gbs


def device_info(torch):
    p = torch.cuda.get_device_properties(0)
    return {"name": p.name, "arch": getattr(p, "gcnArchName", None), "compute_units": p.multi_processor_count,
            "l2_bytes": getattr(p, "L2_cache_size", None), "hbm_bytes": p.total_memory}


def power_law_bench(g2, el2, K, torch):
    """The 41.6M-vertex power-law graph: the plain protocol (300 seeds at k = 1, 2, 10 at k = 3, 6,
    one query per launch sequence, device-resident) and one 256-seed batch at k = 3."""
    import graphgen
    dev = torch.device("cuda:0")
    out = {"graph": "directed Chung-Lu, 41.6M vertices, 1.47B tuples", "vertices": g2.n, "arcs": g2.num_arcs}
    s300 = graphgen.draw_seeds(el2, 300, seed=7, stream=0)
    s10 = graphgen.draw_seeds(el2, 10, seed=7, stream=1)
    tot_te, tot_ms, tot_q = 0, 0.0, 0
    for k, seeds in ((1, s300), (2, s300), (3, s10), (6, s10)):
        d = torch.from_numpy(seeds).to(dev)
        c = torch.empty(len(seeds), dtype=torch.int64, device=dev)
        te = torch.empty(len(seeds), dtype=torch.int64, device=dev)
        for _ in range(2):
            g2.count_dev(d, k, c, te)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        g2.count_dev(d, k, c, te)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        t = int(te.sum())
        lat = []
        for s in seeds[:30]:
            t0 = time.perf_counter()
            g2.count(np.array([s], np.int32), k)
            lat.append((time.perf_counter() - t0) * 1000.0)
        out[f"plain_k{k}"] = {"queries": len(seeds), "ms": round(ms, 3), "qps": round(len(seeds) / (ms / 1e3), 1),
                              "gteps": round(t / (ms / 1e3) / 1e9, 3), "host_api_p50_ms": round(pct(lat, 50), 4),
                              "host_api_p99_ms": round(pct(lat, 99), 4)}
        tot_te += t
        tot_ms += ms
        tot_q += len(seeds)
    out["plain_protocol"] = {"queries": tot_q, "ms": round(tot_ms, 3), "qps": round(tot_q / (tot_ms / 1e3), 1),
                             "gteps": round(tot_te / (tot_ms / 1e3) / 1e9, 3)}
    # per-kernel roles of the deep queries (k = 3 and 6), whose inner hops carry the bytes
    d36 = torch.from_numpy(s10).to(dev)
    c36 = torch.empty(10, dtype=torch.int64, device=dev)
    g2.profile(True)
    for k in (3, 6):
        g2.count_dev(d36, k, c36)
    torch.cuda.synchronize()
    kern = g2.profile_read()
    g2.profile(False)
    empty = kern.pop("empty_launch", None)
    overhead_us = 1000.0 * empty["total_ms"] / empty["launches"] if empty and empty["launches"] else 0.0
    roles = {}
    for name, kv in kern.items():
        avg = max(1000.0 * kv["total_ms"] / max(kv["launches"], 1) - overhead_us, 0.0)
        gbs = kv["algorithmic_bytes"] / kv["launches"] / (avg * 1e-6) / 1e9 if avg > 0 else 0.0
        roles[name] = {"launches": kv["launches"], "avg_us": round(avg, 3), "achieved_gbs": round(gbs, 1),
                       "frac": round(gbs / HBM_PEAK_GBS, 4)}
    out["plain_deep_roles"] = roles
    s256 = graphgen.draw_seeds(el2, 256, seed=13)
    d = torch.from_numpy(s256).to(dev)
    ks = torch.full((256,), 3, dtype=torch.int32, device=dev)
    c = torch.empty(256, dtype=torch.int64, device=dev)
    g2.count_batched_dev(d, ks, c)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    g2.count_batched_dev(d, ks, c)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    dp = torch.empty(256, dtype=torch.int64, device=dev)
    dte = torch.empty(256, dtype=torch.int64, device=dev)
    g2.count_dev(d, 3, dp, dte)
    torch.cuda.synchronize()
    out["batch256_k3"] = {"seeds": 256, "ms": round(ms, 3), "qps": round(256 / (ms / 1e3), 1),
                          "gteps": round(int(dte.sum()) / (ms / 1e3) / 1e9, 3),
                          "equal_to_plain": bool(torch.equal(c, dp))}
    # full-depth breadth-first distances from 8 of the 300 seeds
    deg = g2.degrees()
    d_dist = torch.empty(g2.n, dtype=torch.int32, device=dev)
    d_depth = torch.empty(1, dtype=torch.int32, device=dev)
    bte, bdepth, bms = [], [], []
    for s in s300[:8]:
        g2.bfs_dev(int(s), d_dist, -1, None, d_depth)
        dist = d_dist.cpu().numpy()
        bte.append(int(deg[dist >= 0].sum()))
        bdepth.append(int(d_depth.item()))
        e0.record()
        g2.bfs_dev(int(s), d_dist, -1)
        e1.record()
        e1.synchronize()
        bms.append(e0.elapsed_time(e1))
    out["bfs"] = {"seeds": 8, "ms_per_search": round(float(np.mean(bms)), 3), "p50_ms": round(pct(bms, 50), 3),
                  "gteps": round(sum(bte) / (sum(bms) / 1e3) / 1e9, 2), "depth_mean": round(float(np.mean(bdepth)), 2),
                  "teps_edges": "stored out-arcs of every reached vertex"}
    log("power-law graph: " + json.dumps(out))
    return out


def bfs_bench(g, el, K, torch, n_seeds=64, cpu_leg=True):
    """Full-depth breadth-first distances (no depth limit) from sampled seeds,
    device-resident, through khop_bfs_dev on one stream."""
    import graphgen
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    seeds = graphgen.draw_seeds(el, n_seeds, seed=7, stream=2)
    deg = g.degrees()
    d_dist = torch.empty(g.n, dtype=torch.int32, device=dev)
    d_count = torch.empty(1, dtype=torch.int64, device=dev)
    d_depth = torch.empty(1, dtype=torch.int32, device=dev)
    # untimed pass: the traversed edges (out-arcs of every reached vertex), depth and reach of each search
    te, depth, reach = [], [], []
    for s in seeds:
        g.bfs_dev(int(s), d_dist, -1, d_count, d_depth, stream=stream)
        dist = d_dist.cpu().numpy()
        te.append(int(deg[dist >= 0].sum()))
        depth.append(int(d_depth.item()))
        reach.append(int(d_count.item()) + 1)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ms = []
    t0 = time.perf_counter()
    for s in seeds:
        ev[0].record(stream)
        g.bfs_dev(int(s), d_dist, -1, d_count, d_depth, stream=stream)
        ev[1].record(stream)
        ev[1].synchronize()
        ms.append(ev[0].elapsed_time(ev[1]))
    wall = time.perf_counter() - t0
    # per-kernel times of the same searches
    g.profile(True)
    for s in seeds[:16]:
        g.bfs_dev(int(s), d_dist, -1, d_count, d_depth, stream=stream)
    torch.cuda.synchronize()
    kern = g.profile_read()
    g.profile(False)
    empty = kern.pop("empty_launch", None)
    overhead_us = 1000.0 * empty["total_ms"] / empty["launches"] if empty and empty["launches"] else 0.0
    kinds = {}
    for name, kv in kern.items():
        avg = max(1000.0 * kv["total_ms"] / max(kv["launches"], 1) - overhead_us, 0.0)
        kinds[name] = {"launches_per_search": round(kv["launches"] / 16, 2), "avg_us": round(avg, 3),
                       "gbs": round(kv["algorithmic_bytes"] / kv["launches"] / (avg * 1e-6) / 1e9, 1)
                       if avg > 0 else 0}
    tot_te = sum(te)
    out = {"seeds": len(seeds), "max_depth": "none", "ms_per_search": round(float(np.mean(ms)), 4),
           "p50_ms": round(pct(ms, 50), 4), "p99_ms": round(pct(ms, 99), 4),
           "searches_per_s": round(len(seeds) / wall, 1),
           "gteps": round(tot_te / (sum(ms) / 1e3) / 1e9, 2),
           "teps_edges": "stored out-arcs of every reached vertex (each undirected edge twice)",
           "depth_mean": round(float(np.mean(depth)), 2), "depth_max": int(max(depth)),
           "reach_mean": round(float(np.mean(reach)), 1), "kernels": kinds}
    log(f"bfs: {out['ms_per_search']} ms per search, {out['gteps']} GTEPS, depth {out['depth_mean']}")
    if cpu_leg:
        import oracle
        og = oracle.OracleGraph.from_edgelist(el)
        c_ms, equal = [], True
        for i, s in enumerate(seeds[:2]):
            t = time.perf_counter()
            ref = og.distances(int(s), 2**31 - 1)
            c_ms.append((time.perf_counter() - t) * 1000.0)
            g.bfs_dev(int(s), d_dist, -1, stream=stream)
            equal = equal and bool(np.array_equal(d_dist.cpu().numpy(), ref))
        out["cpu_oracle"] = {"searches": 2, "cores": 1, "ms_per_search": round(float(np.mean(c_ms)), 1),
                             "gteps": round(sum(te[:2]) / (sum(c_ms) / 1e3) / 1e9, 4), "distances_equal_gpu": equal}
    return out


def sets_bench(g, el, groups, K, torch, cpu_leg=True):
    """The k = 2 neighborhoods of the protocol's 300 k = 2 seeds returned as
    vertex ids (device-resident and through the host entry point), and the
    exactly-l level sizes of its 10 k = 6 seeds."""
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    seeds = dict(groups)[2]
    deep = dict(groups)[6]
    d_ids = torch.empty(g.n, dtype=torch.int32, device=dev)
    d_count = torch.empty(1, dtype=torch.int64, device=dev)
    d_lv = torch.empty(6, dtype=torch.int64, device=dev)
    sizes = []
    for s in seeds:
        g.neighborhood_dev(int(s), 2, d_ids, d_count, stream=stream)
        sizes.append(int(d_count.item()))
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    torch.cuda.synchronize()
    ev[0].record(stream)
    for s in seeds:
        g.neighborhood_dev(int(s), 2, d_ids, d_count, stream=stream)
    ev[1].record(stream)
    ev[1].synchronize()
    dev_ms = ev[0].elapsed_time(ev[1]) / len(seeds)
    ev[0].record(stream)
    for s in deep:
        g.levels_dev(int(s), 6, d_lv, stream=stream)
    ev[1].record(stream)
    ev[1].synchronize()
    lv_ms = ev[0].elapsed_time(ev[1]) / len(deep)
    # the set kernels' own time and bytes
    g.profile(True)
    for s in seeds[:32]:
        g.neighborhood_dev(int(s), 2, d_ids, d_count, stream=stream)
    torch.cuda.synchronize()
    kern = g.profile_read()
    g.profile(False)
    empty = kern.pop("empty_launch", None)
    overhead_us = 1000.0 * empty["total_ms"] / empty["launches"] if empty and empty["launches"] else 0.0
    st = kern.get("plain_set", {"launches": 0})
    set_us = max(1000.0 * st["total_ms"] / st["launches"] - overhead_us, 0.0) if st["launches"] else 0.0
    set_gbs = st["algorithmic_bytes"] / st["launches"] / (set_us * 1e-6) / 1e9 if set_us > 0 else 0.0
    # through the host entry point: ids copied to host memory
    host = []
    for s in seeds[:100]:
        t = time.perf_counter()
        ids = g.neighborhood(int(s), 2)
        host.append((time.perf_counter() - t) * 1000.0)
    out = {"k": 2, "seeds": len(seeds), "ids_mean": round(float(np.mean(sizes)), 1), "ids_max": int(max(sizes)),
           "device_ms_per_query": round(dev_ms, 4),
           "device_ids_per_s": round(float(np.sum(sizes)) / (dev_ms * len(seeds) / 1e3), 1),
           "set_kernels": {"avg_us": round(set_us, 3), "gbs": round(set_gbs, 1),
                           "bytes": "visited bitmap read twice, block counts, 4 B per id written"},
           "host_api_p50_ms": round(pct(host, 50), 4), "host_api_p99_ms": round(pct(host, 99), 4),
           "levels_k6_ms_per_query": round(lv_ms, 4)}
    log(f"sets: k=2 {out['ids_mean']} ids per query, {out['device_ms_per_query']} ms device, "
        f"{out['host_api_p50_ms']} ms host p50; set kernels {out['set_kernels']}")
    if cpu_leg:
        import oracle
        og = oracle.OracleGraph.from_edgelist(el)
        equal = True
        for s in seeds[:3]:
            d = og.distances(int(s), 2)
            equal = equal and bool(np.array_equal(g.neighborhood(int(s), 2), np.nonzero(d >= 1)[0]))
        for s in deep[:2]:
            equal = equal and bool(np.array_equal(g.levels(int(s), 6), og.khop(int(s), 6)[2]))
        out["equal_oracle"] = equal
    return out


def filtered_bench(g, el, groups, K, torch, cpu_leg=True):
    """The protocol's query set counted in the subgraph of a random half of the
    vertices (a vertex-label filter), device-resident, one launch sequence per query."""
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    lab = np.random.default_rng(2024).random(g.n) < 0.5
    d_bits = torch.from_numpy(K.label_bits(lab, g.n).view(np.int64)).to(dev)
    runs = []
    for k, seeds in groups:
        ds = torch.from_numpy(seeds).to(dev)
        dc = torch.empty(len(seeds), dtype=torch.int64, device=dev)
        dt = torch.empty(len(seeds), dtype=torch.int64, device=dev)
        runs.append((k, seeds, ds, dc, dt))

    def one_pass():
        for k, _, ds, dc, dt in runs:
            g.count_labeled_dev(ds, k, d_bits, dc, dt, stream=stream)

    for _ in range(2):
        one_pass()
    torch.cuda.synchronize()
    te = sum(int(dt.sum()) for *_, dt in runs)
    nq = sum(len(s) for _, s, *_ in runs)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record(stream)
    for _ in range(5):
        one_pass()
    ev[1].record(stream)
    ev[1].synchronize()
    ms = ev[0].elapsed_time(ev[1]) / 5
    out = {"label_density": 0.5, "queries": nq, "ms_per_pass": round(ms, 3), "qps": round(nq / (ms / 1e3), 1),
           "gteps": round(te / (ms / 1e3) / 1e9, 2)}
    # the same queries as one batched call (host entry point: mask and seeds copied in, counts out)
    all_seeds = np.concatenate([s for _, s, *_ in runs]).astype(np.int32)
    all_ks = np.concatenate([np.full(len(s), k, np.int32) for k, s, *_ in runs])
    plain_counts = np.concatenate([dc.cpu().numpy() for *_, dc, _ in runs])
    b = g.count_batched_labeled(all_seeds, all_ks, lab)
    t = time.perf_counter()
    for _ in range(5):
        b = g.count_batched_labeled(all_seeds, all_ks, lab)
    bms = (time.perf_counter() - t) * 1000.0 / 5
    out["batched"] = {"ms_per_pass_host": round(bms, 3), "qps": round(nq / (bms / 1e3), 1),
                      "equal_to_plain": bool(np.array_equal(b, plain_counts))}
    log(f"label-filtered protocol: {out['ms_per_pass']} ms per {nq} queries, {out['gteps']} GTEPS; "
        f"batched {out['batched']}")
    if cpu_leg:
        import oracle
        og = oracle.OracleGraph.from_edgelist(el)
        equal = True
        for k, seeds, ds, dc, dt in runs:
            got = dc.cpu().numpy()
            for i in range(0, len(seeds), max(1, len(seeds) // 5)):
                equal = equal and og.khop_filtered(int(seeds[i]), k, lab.astype(np.uint8))[0] == int(got[i])
        out["sample_equal_oracle"] = bool(equal)
    return out


def copy_calibration(nbytes=256 << 20, reps=5):
    """Device-to-device copies of a known size: under rocprofv3 --pmc their FETCH_SIZE and
    WRITE_SIZE per dispatch give the factor between the counters and bytes moved."""
    import torch
    a = torch.ones(nbytes // 4, dtype=torch.int32, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes": nbytes, "dispatches": reps}), flush=True)


def batched_sweep(g, el, K, torch):
    """One 1024-seed draw answered at k = 3 and 6 with 64, 256 and 1024 seeds per batched launch (the same
    queries each time, so the figures differ by the batch width only), beside the plain path."""
    import graphgen
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    s1024 = graphgen.draw_seeds(el, 1024, seed=11)
    d_s = torch.from_numpy(s1024).to(dev)
    d_te = torch.empty(1024, dtype=torch.int64, device=dev)
    d_c = torch.empty(1024, dtype=torch.int64, device=dev)
    d_b = torch.empty(1024, dtype=torch.int64, device=dev)
    saved = g.get_option(K.KHOP_OPT_BATCH_SEEDS)
    out = {"seeds": 1024, "note": "the same 1024 queries at every batch width"}
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for k in (3, 6):
        g.count_dev(d_s, k, d_c, d_te, stream=stream)  # plain path: per-seed traversed edges
        torch.cuda.synchronize()
        te = float(d_te.cpu().numpy().sum())
        plain_counts = d_c.cpu().numpy()
        for _ in range(2):
            g.count_dev(d_s, k, d_c, stream=stream)
        e0.record(stream)
        g.count_dev(d_s, k, d_c, stream=stream)
        e1.record(stream)
        e1.synchronize()
        plain_ms = e0.elapsed_time(e1)
        out[f"plain_k{k}"] = {"ms": round(plain_ms, 3), "qps": round(1024 / (plain_ms / 1e3), 1),
                              "gteps": round(te / (plain_ms / 1e3) / 1e9, 2)}
        d_k = torch.full((1024,), k, dtype=torch.int32, device=dev)
        for per in (64, 256, 1024):
            g.set_option(K.KHOP_OPT_BATCH_SEEDS, per)
            g.count_batched_dev(d_s, d_k, d_b, stream=stream)
            torch.cuda.synchronize()
            if not np.array_equal(d_b.cpu().numpy(), plain_counts):
                raise SystemExit(f"batched counts differ from plain ({per} seeds per launch, k={k})")
            reps = 3
            e0.record(stream)
            for _ in range(reps):
                g.count_batched_dev(d_s, d_k, d_b, stream=stream)
            e1.record(stream)
            e1.synchronize()
            ms = e0.elapsed_time(e1) / reps
            out[f"batch{per}_k{k}"] = {"seeds_per_launch": per, "ms": round(ms, 3),
                                       "qps": round(1024 / (ms / 1e3), 1), "gteps": round(te / (ms / 1e3) / 1e9, 2)}
    g.set_option(K.KHOP_OPT_BATCH_SEEDS, saved)
    log("batched sweep: " + ", ".join(f"{k}={v['qps']} q/s" for k, v in out.items() if isinstance(v, dict)))
    return out


def _lane_delta(before, after):
    """Per-lane counters accumulated between two khop_server_stats snapshots."""
    out = {}
    for b0, a0 in zip(before, after):
        n = a0["launches"] - b0["launches"]
        q = a0["queries"] - b0["queries"]
        ms = a0["busy_ms"] - b0["busy_ms"]
        out[f"g{a0['graph_id']}_{a0['lane']}"] = {
            "launches": n, "queries": q, "queries_per_launch": round(q / n, 1) if n else 0,
            "ms_per_launch": round(ms / n, 3) if n else 0, "words_held": a0["words"]}
    return out


def serving_bench(K, graphs, seconds):
    """Open-loop Poisson arrivals at 0.25, 0.5 and 0.8 of the closed-loop saturation rate, at least
    10^4 queries per level.

    Queries: k in {1, 2, 3, 6} with weights 0.4/0.3/0.2/0.1, seeds uniform over
    non-isolated vertices, graph uniform over the resident graphs.  Latency is
    completion minus scheduled arrival (CLOCK_MONOTONIC).
    """
    import threading

    import graphgen
    rng = np.random.default_rng(2024)
    pools = [graphgen.draw_seeds(el, 50000, seed=21) for _, _, el in graphs]
    names = [name for name, _, _ in graphs]

    def make(n):
        gi = rng.integers(0, len(graphs), size=n)
        ks = rng.choice(np.array([1, 2, 3, 6]), size=n, p=[0.4, 0.3, 0.2, 0.1])
        si = rng.integers(0, 50000, size=n)
        return [(int(a), int(pools[a][b]), int(c)) for a, b, c in zip(gi, si, ks)]

    def collect(srv, n, deadline_s=120.0):
        got = {}
        t_end = time.time() + deadline_s
        while len(got) < n and time.time() < t_end:
            for r in srv.poll(8192):
                got[r.ticket] = r
            time.sleep(0.0005)
        return got

    def closed_loop(srv, ids, window=2048, seconds=1.5):
        """Saturation: `window` requests kept outstanding (a completed one is replaced at once) for
        `seconds` after a warm-up of the same length; completed requests per second."""
        outstanding = 0
        done = 0
        t_end = None
        t_warm = time.perf_counter() + seconds
        t0 = None
        while True:
            if outstanding < window:
                for gi, sd, k in make(window - outstanding):
                    srv.submit(ids[gi], sd, k)
                outstanding = window
            got = srv.poll(8192)
            outstanding -= len(got)
            now = time.perf_counter()
            if t0 is None and now >= t_warm:
                t0, t_end = now, now + seconds
            elif t0 is not None:
                done += len(got)
                if now >= t_end:
                    break
            if not got:
                time.sleep(0.0002)
        rate = done / (time.perf_counter() - t0)
        srv.drain(120000)
        srv.poll(1 << 20)
        return rate

    srv = K.Server(96 << 30, 1024)
    ids = [srv.add_graph(g) for _, g, _ in graphs]
    srv.set_option(K.KHOP_SERVER_ROUTE, K.KHOP_ROUTE_BATCH)
    sat_batch = closed_loop(srv, ids)
    srv.set_option(K.KHOP_SERVER_ROUTE, K.KHOP_ROUTE_AUTO)
    sat = closed_loop(srv, ids)
    log(f"serving {'+'.join(names)}: closed loop {sat:.0f} queries/s (batch lanes only: {sat_batch:.0f})")
    levels = []
    check = []
    import gc
    gc.collect()
    gc.disable()  # a collector pause in the producer thread would delay arrivals
    for frac in (0.25, 0.5, 0.8):
        qps = frac * sat
        n = int(min(max(qps * seconds, 10000), 60000))  # at least 10^4 queries per level
        qs = make(n)
        gaps = rng.exponential(1.0 / qps, size=n)
        sched = np.cumsum(gaps)
        tick = {}
        st0 = srv.stats()
        t_base = K.monotonic_ns() + 2_000_000

        def producer():
            for i, (gi, sd, k) in enumerate(qs):
                due = t_base + int(sched[i] * 1e9)
                while K.monotonic_ns() < due:
                    pass
                tick[srv.submit(ids[gi], sd, k)] = (due, i)

        th = threading.Thread(target=producer)
        th.start()
        th.join()
        got = collect(srv, n)
        st1 = srv.stats()
        lat = []
        by_gk = {}
        single = 0
        done_last = 0
        for t, (due, i) in tick.items():
            r = got.get(t)
            if r is None or r.status != K.KHOP_OK:
                continue
            ms = (r.t_done_ns - due) / 1e6
            lat.append(ms)
            single += r.path == K.KHOP_PATH_SINGLE
            by_gk.setdefault(f"{names[qs[i][0]]}_k{qs[i][2]}", []).append(ms)
            done_last = max(done_last, r.t_done_ns)
            if len(check) < 400 and i % 25 == 0:
                check.append((qs[i], r.count))
        span = (done_last - t_base) / 1e9 if done_last else float("nan")
        offered_span = float(sched[-1])
        # served rate in steady state: completions within the middle 80% of the arrival window (the
        # first and last tenth hold the ramp-up and the drain of the last arrivals)
        lo, hi = t_base + int(0.1 * offered_span * 1e9), t_base + int(0.9 * offered_span * 1e9)
        mid = sum(1 for t in tick if t in got and got[t].status == K.KHOP_OK and lo <= got[t].t_done_ns < hi)
        levels.append({"offered_qps": round(qps, 1), "achieved_qps": round(mid / (0.8 * offered_span), 1),
                       "completed_over_full_span_qps": round(len(lat) / span, 1),
                       "arrival_span_s": round(offered_span, 3), "completion_span_s": round(span, 3),
                       "n": n, "completed": len(lat), "p50_ms": round(pct(lat, 50), 3),
                       "p99_ms": round(pct(lat, 99), 3), "max_ms": round(float(np.max(lat)), 3),
                       "mean_ms": round(float(np.mean(lat)), 3),
                       "single_query_share": round(single / max(len(lat), 1), 3),
                       "lanes": _lane_delta(st0, st1),
                       "by_graph_k": {key: {"n": len(v), "mean_ms": round(float(np.mean(v)), 3),
                                            "p50_ms": round(pct(v, 50), 3), "p99_ms": round(pct(v, 99), 3)}
                                      for key, v in sorted(by_gk.items())}})
        log(f"serving {'+'.join(names)} at {qps:.0f} q/s offered: {levels[-1]['achieved_qps']:.0f} served, "
            f"p50 {levels[-1]['p50_ms']} ms, p99 {levels[-1]['p99_ms']} ms")
    gc.enable()
    srv.close()
    # served counts against the plain path, query by query
    ok = 0
    for (gi, sd, k), c in check:
        ok += int(graphs[gi][1].count(np.array([sd], np.int32), k)[0] == c)
    return {"graphs": names, "k_weights": {"1": 0.4, "2": 0.3, "3": 0.2, "6": 0.1},
            "max_batch_seeds": 1024, "saturation_qps": round(sat, 1), "saturation_qps_batch_lanes_only":
            round(sat_batch, 1), "saturation": "completions per second with 2048 requests kept outstanding",
            "levels": levels, "checked_against_plain": len(check), "equal": ok}


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
