"""Benchmark of the randomized level push on one MI355X.

Default workload (one step = one pass of the whole hot path over one batch):
  R-MAT graph, scale 22 (4,194,304 nodes), 16 generated edges per node,
  (a, b, c) = (0.57, 0.19, 0.19), symmetrised, deduplicated, loops dropped;
  256 sources drawn uniformly among nodes of degree >= 1;
  * Katz: a = b = 0, w_i = 0.85 beta^i with beta = 0.85 / lambda_1 (lambda_1 by
    FP64 power iteration), L = 30, eps = 1e-7, the 256 sources in one call;
  * 10-step transition probability: a = 0, b = 1, w_10 = 1, L = 10,
    eps = 1e-7, the same 256 sources in one call.
The value is edge pushes (deterministic + accepted sampled pushes, the cost
unit of Theorem 3.3) per second over the timed steps, inputs resident in HBM.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
METRIC = "edge-pushes/s + HBM GB/s; queries/s and p99 latency batched vs per-query at eps"


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def alg_bytes(st: dict, levels, a_zero: bool) -> float:
    """Algorithmic bytes of the given level launches: 16 B per frontier
    (node, column) entry (residue read, reserve read-modify-write, clear),
    12 B per edge push (neighbour id + residue read-modify-write; 16 B when
    a != 0 for the degree factor), 8 B per rejected candidate."""
    b_push = 12.0 if a_zero else 16.0
    tot = 0.0
    for i in levels:
        pushes = float(st["det"][i]) + float(st["acc"][i])
        rejected = float(st["cand"][i]) - float(st["acc"][i])
        tot += 16.0 * float(st["frontier"][i]) + b_push * pushes + 8.0 * rejected
    return tot


def build_workload(log_fn, cache_dir):
    from paper_2106_03058_amd import inputs

    path = os.path.join(cache_dir, "rmat22_ef16_s2.npz") if cache_dir else None
    t = time.time()
    if path and os.path.exists(path):
        z = np.load(path)
        g = inputs.Graph(int(z["n"]), z["row_ptr"], z["col"])
        lam = float(z["lam"])
        log_fn(f"graph and lambda_1 loaded from {path} in {time.time() - t:.1f}s")
    else:
        g = inputs.rmat(22, 16, 0.57, 0.19, 0.19, seed=2)
        log_fn(f"graph {g.describe()} in {time.time() - t:.1f}s")
        t = time.time()
        lam = inputs.lambda_max(g, tol=1e-10, max_iter=1000)
        log_fn(f"lambda_1 = {lam:.6f} in {time.time() - t:.1f}s")
        if path:
            os.makedirs(cache_dir, exist_ok=True)
            np.savez(path, n=g.n, row_ptr=g.row_ptr, col=g.col, lam=lam)
    beta = 0.85 / lam
    src = inputs.sources_uniform(g, 256, seed=102)
    katz = dict(name="katz", a=0.0, b=0.0, w=inputs.weights_katz(beta, 30, 0.85), eps=1e-7,
                qids=np.arange(256, dtype=np.uint32))
    tp = dict(name="tp", a=0.0, b=1.0, w=inputs.weights_tp(10), eps=1e-7,
              qids=np.arange(256, 512, dtype=np.uint32))
    return g, src, [katz, tp], lam


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--seed", type=int, default=2021)
    ap.add_argument("--single", type=int, default=16, help="queries timed one per launch")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-queries", type=int, default=4, help="oracle sample per model")
    ap.add_argument("--cache", default=os.environ.get("AGP_BENCH_CACHE", ""),
                    help="directory to keep the generated graph between runs")
    ap.add_argument("--models", default="katz,tp", help="subset of the step to run (profiling)")
    ap.add_argument("--columns", type=int, default=256, help="queries per call (profiling)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="copy 1 GiB device to device first (reference for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        return 2

    import torch

    from paper_2106_03058_amd import agp

    agp.lib()
    dev = torch.device("cuda:0")
    g, src, models, lam = build_workload(log, args.cache)
    keep = set(args.models.split(","))
    models = [m for m in models if m["name"] in keep]
    src = src[: args.columns]
    for m in models:
        m["qids"] = m["qids"][: args.columns]
    if args.calibrate_copy:
        a = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        b_ = torch.empty_like(a)
        b_.copy_(a)
        torch.cuda.synchronize()
        del a, b_
    t = time.time()
    G = agp.Graph.from_inputs(g)
    torch.cuda.synchronize()
    log(f"device graph build (degree sort) {time.time() - t:.2f}s, max degree {G.max_degree}")
    C = src.size
    X = torch.zeros((g.n, C), dtype=torch.float32, device=dev)
    X[torch.from_numpy(src).to(dev), torch.arange(C, device=dev)] = 1.0
    outs = [torch.empty_like(X) for _ in models]

    def step(stats: bool):
        res = []
        for m, o in zip(models, outs):
            t0 = time.perf_counter()
            _, st = agp.propagate(G, m["a"], m["b"], m["w"], X, m["eps"], args.seed, qids=m["qids"],
                                  out=o, stats=stats)
            res.append((st, (time.perf_counter() - t0) * 1e3))
        return res

    for _ in range(args.warmup):
        step(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    runs = [step(True) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    pushes_step = sum(st["pushes"] for st, _ in runs[0])
    for r in runs[1:]:  # identical seeds: identical work every step
        assert sum(st["pushes"] for st, _ in r) == pushes_step
    value = pushes_step / (ms_per_step / 1e3)
    log(f"{ms_per_step:.1f} ms/step, {pushes_step:.3e} pushes/step")

    # roofline of the dominant kernel: the level kernel of the middle levels
    mid_bytes = mid_ms = 0.0
    launches = 0
    all_bytes = all_ms = 0.0
    for r in runs:
        for (st, _), m in zip(r, models):
            L = st["levels"]
            mids = range(1, L)
            mid_bytes += alg_bytes(st, mids, m["a"] == 0.0)
            mid_ms += float(st["level_ms"][1:L].sum())
            launches += max(L - 1, 0)
            all_bytes += alg_bytes(st, range(L + 1), m["a"] == 0.0)
            all_ms += float(st["level_ms"].sum())
    achieved = mid_bytes / (mid_ms / 1e3) / 1e9
    per_level = []
    for (st, ms), m in zip(runs[0], models):
        per_level.append({"model": m["name"], "call_ms": round(ms, 3),
                          "frontier": [int(v) for v in st["frontier"]],
                          "pushes": [int(d + a) for d, a in zip(st["det"], st["acc"])],
                          "level_ms": [round(float(v), 4) for v in st["level_ms"]]})

    # batched vs one query per launch, same eps and keys (identical results)
    lat_b = []
    for (st, ms), m in zip(runs[-1], models):
        lat_b += [ms] * C
    lat_b = np.array(lat_b)
    q_per_s_batched = len(models) * C / (ms_per_step / 1e3)
    lat_s = []
    nq = args.single // len(models)
    one = torch.empty((g.n, 1), dtype=torch.float32, device=dev)
    single_ok = True
    for m, o in zip(models, outs):
        for c in range(nq):
            xc = X[:, c:c + 1].contiguous()
            torch.cuda.synchronize()
            ts = time.perf_counter()
            agp.propagate(G, m["a"], m["b"], m["w"], xc, m["eps"], args.seed, qids=m["qids"][c:c + 1], out=one)
            lat_s.append((time.perf_counter() - ts) * 1e3)
            single_ok &= bool(torch.equal(one[:, 0], o[:, c]))
    lat_s = np.array(lat_s) if lat_s else np.zeros(1)
    q_per_s_single = 1e3 / lat_s.mean() if lat_s.any() else 0.0

    result = {
        "metric": METRIC,
        "value": value,
        "unit": "edge-pushes/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "+".join(m["name"] for m in models) + f", {C} sources each, rmat scale 22",
            "graph": g.describe(),
            "models": {m["name"]: {"a": m["a"], "b": m["b"], "L": len(m["w"]) - 1, "eps": m["eps"]} for m in models},
            "lambda_1": lam,
            "columns_per_call": C,
        },
        "pushes_per_step": pushes_step,
        "hbm_gbps_algorithmic_all_levels": all_bytes / (all_ms / 1e3) / 1e9,
        "queries_per_s_batched": q_per_s_batched,
        "latency_ms_batched": {"p50": float(np.percentile(lat_b, 50)), "p99": float(np.percentile(lat_b, 99))},
        "queries_per_s_one_per_launch": q_per_s_single,
        "latency_ms_one_per_launch": {"p50": float(np.percentile(lat_s, 50)),
                                      "p99": float(np.percentile(lat_s, 99)), "queries": int(lat_s.size)},
        "one_per_launch_equals_batched": single_ok,
        "roofline": {
            "bound": "hbm",
            "kernel": "k_level<float, false, false> (levels 1..L-1)",
            "achieved": achieved,
            "peak": HBM_PEAK_GBPS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBPS,
            "traffic": None,
            "avg_launch_ms": mid_ms / max(launches, 1),
            "alg_bytes_per_launch": mid_bytes / max(launches, 1),
        },
        "per_level": per_level,
    }

    if not args.no_cpu_baseline:
        import oracle

        k = args.cpu_queries
        threads = min(2 * k, 16, os.cpu_count() or 1)
        t = time.time()
        sg = oracle.degree_sort(g)
        log(f"oracle degree sort {time.time() - t:.1f}s")
        cols = np.arange(k)
        tot_push = 0
        parity = True
        t = time.time()
        xs = np.zeros((g.n, k), dtype=np.float32)
        xs[src[cols], np.arange(k)] = 1.0
        import threading

        results = {}

        def run(mi, m):
            results[mi] = oracle.propagate(sg, m["a"], m["b"], m["w"], xs, m["eps"], args.seed,
                                           qids=m["qids"][cols], threads=max(threads // len(models), 1))

        ths = [threading.Thread(target=run, args=(mi, m)) for mi, m in enumerate(models)]
        for th in ths:
            th.start()
        for th in ths:
            th.join()
        wall = time.time() - t
        for mi, m in enumerate(models):
            ref, cnt = results[mi]
            tot_push += int(cnt["det"].sum() + cnt["acc"].sum())
            got = outs[mi][:, :k].cpu().numpy().astype(np.float64)
            parity &= bool(np.array_equal(got, ref))
        log(f"oracle sample {wall:.1f}s, parity {parity}")
        result["cpu_baseline"] = {
            "value": tot_push / wall,
            "unit": "edge-pushes/s",
            "cores": threads,
            "kind": "oracle",
            "sample": f"{k} Katz + {k} TP queries (first {k} sources, same seeds), {wall:.1f}s wall",
        }
        result["parity_full_size"] = {"columns_checked": 2 * k, "bit_exact": parity}
    print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
