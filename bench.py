"""Benchmark of the randomized level push on one MI355X.

Default workload, `--workload gnn-ppr-large` (one step = one pass of the
whole hot path over one batch): PPR feature propagation (alpha = 0.1,
L = 10, a = b = 1/2, eps = 1e-8) of a 111,059,956 x 128 U[-1, 1] binary32
feature matrix on a Chung-Lu graph (n = 111,059,956, exponent 2.2, ~1.6e9
arcs plus one loop per node) generated on the GPU; graph and features stay
resident in HBM, the 128 columns run as tiles of node-major dense levels.
Other workloads:
  `--workload katz-tp`: R-MAT graph, scale 22 (4,194,304 nodes), 16
    generated edges per node, (a, b, c) = (0.57, 0.19, 0.19), symmetrised,
    deduplicated, loops dropped; 256 sources drawn uniformly among nodes of
    degree >= 1; Katz (a = b = 0, w_i = 0.85 beta^i, beta = 0.85 / lambda_1,
    L = 30, eps = 1e-7) and 10-step transition probability (a = 0, b = 1,
    w_10 = 1, eps = 1e-7), the 256 sources in one call each.
  `--workload gnn-hkpr`: heat-kernel feature propagation (t = 5, L = 10,
    a = b = 1/2, eps = 1e-7) of a 2.4M x 128 N(0,1) matrix on a Chung-Lu
    graph (n = 2.4M, mean degree 50, exponent 2.5, one self-loop per node).
  `--workload serve`: a served query stream on R-MAT scale 24.
  `--workload cluster`: local clustering, heat kernel PageRank (t = 5,
    L = 20, eps = 1e-7) from 64 seeds and the minimum-conductance sweep of
    each, on an Orkut-shaped Chung-Lu graph (3.07M nodes, 117M edges).
  `--workload variants`: the paper-literal x+/x- split and infinite-tail
    Y_i against the defaults (time, pushes, error against the exact sum).
  `--workload directed`: PPR from 256 sources along out-edges and
    single-target PPR to 256 targets along in-edges (alpha = 0.2, L = 20,
    eps = 1e-7) on a directed R-MAT scale 22 (arcs as generated).
The value is edge pushes (deterministic + accepted sampled pushes, the cost
unit of Theorem 3.3) per second over the timed steps, inputs resident in HBM.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import threading
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
# Vector ALU issue rate of MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
# = 39.32e12 lane-instructions/s (32-bit integer, binary32 and binary64
# adds/multiplies/FMAs all issue at this rate on gfx950).  One random draw of
# the sampling step is at least 103 such instructions: Philox4x32-10 (42,
# with 32x32->64 multiply-adds), two 53-bit uniforms and the 7-step lifted
# geometric skip (61), counted in the gfx950 assembly of a draw-only loop;
# the skip table of each run, the acceptance test of each candidate and every
# memory access come on top.  A level whose time goes to its draws is bound
# by ALU_PEAK_DRAWS draws/s.
VALU_LANE_OPS = 256 * 4 * 16 * 2.4e9
VALU_PER_DRAW = 103
ALU_PEAK_GDRAWS = VALU_LANE_OPS / VALU_PER_DRAW / 1e9

# HBM bytes per launch of the level kernel (levels 1..L with the launches
# that make its deferred rows and suffixes), from two rocprofv3 --pmc runs
# of this script (FETCH_SIZE, then WRITE_SIZE) with --calibrate-copy;
# FETCH_SIZE is scaled by 2.0, the factor that makes the 1 GiB copy read
# 1 GiB (WRITE_SIZE reads 1 GiB as written).  Valid only for the kernel
# sources they were taken from (the files that define k_level, k_det_big and
# k_samp_big, code without comments) and the default tuning.
TRAFFIC = {
    "gnn-ppr-large": {"sources": "0fd3ed3950369b42", "columns": 128, "bytes_per_launch": 102346960000.0,
                      "fetch_bytes": 85478380000.0, "write_bytes": 16868580000.0},
}
KERNEL_SOURCES = ("paper_2106_03058_amd/csrc/level_kernels.h", "paper_2106_03058_amd/csrc/agp_device.h")


def _code_only(text: str) -> str:
    """C++ source without its comments and with whitespace runs collapsed, so
    that a comment edit does not retire a traffic record."""
    out, i, n = [], 0, len(text)
    while i < n:
        ch = text[i]
        if ch in "\"'":  # string or character literal: copied as it is
            j = i + 1
            while j < n and text[j] != ch:
                j += 2 if text[j] == "\\" else 1
            out.append(text[i:j + 1])
            i = j + 1
        elif text.startswith("//", i):
            j = text.find("\n", i)
            i = n if j < 0 else j
        elif text.startswith("/*", i):
            j = text.find("*/", i + 2)
            i = n if j < 0 else j + 2
        else:
            out.append(ch)
            i += 1
    return " ".join("".join(out).split())


def kernel_sources_sha() -> str:
    import hashlib

    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), encoding="utf-8") as fh:
            h.update(_code_only(fh.read()).encode())
    return h.hexdigest()[:16]


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


def cached(cache_dir, name, make):
    """Generated inputs, kept in cache_dir between runs of one session."""
    from paper_2106_03058_amd import inputs

    path = os.path.join(cache_dir, name + ".npz") if cache_dir else None
    t = time.time()
    if path and os.path.exists(path):
        z = np.load(path)
        g = inputs.Graph(int(z["n"]), z["row_ptr"], z["col"])
        extra = {k: z[k] for k in z.files if k not in ("n", "row_ptr", "col")}
        log(f"{name} loaded from cache in {time.time() - t:.1f}s")
        return g, extra
    g, extra = make()
    log(f"{name}: {g.describe()} in {time.time() - t:.1f}s")
    if path:
        os.makedirs(cache_dir, exist_ok=True)
        np.savez(path, n=g.n, row_ptr=g.row_ptr, col=g.col, **extra)
    return g, extra


def host_workload(g, signal, models, cfg, unit):
    """A workload whose graph and signal are generated on the host."""
    import torch

    from paper_2106_03058_amd import agp

    state = {}

    def make_graph():
        return agp.Graph.from_inputs(g)

    def signal_device():
        state["x"] = signal()
        return torch.from_numpy(state["x"]).to("cuda:0")

    def oracle_inputs(cols):
        return g, np.ascontiguousarray(state["x"][:, cols])

    return dict(n=g.n, make_graph=make_graph, signal_device=signal_device, models=models, cfg=cfg, unit=unit,
                oracle_inputs=oracle_inputs)


def workload_katz_tp(args):
    from paper_2106_03058_amd import inputs

    def make():
        g = inputs.rmat(22, 16, 0.57, 0.19, 0.19, seed=2)
        t = time.time()
        lam = inputs.lambda_max(g, tol=1e-10, max_iter=1000)
        log(f"lambda_1 = {lam:.6f} in {time.time() - t:.1f}s")
        return g, {"lam": np.array(lam)}

    g, extra = cached(args.cache, "rmat22_ef16_s2", make)
    lam = float(extra["lam"])
    beta = 0.85 / lam
    src = inputs.sources_uniform(g, 256, seed=102)[: args.columns]
    C = src.size
    models = [
        dict(name="katz", a=0.0, b=0.0, w=inputs.weights_katz(beta, 30, 0.85), eps=1e-7,
             qids=np.arange(C, dtype=np.uint32)),
        dict(name="tp", a=0.0, b=1.0, w=inputs.weights_tp(10), eps=1e-7,
             qids=np.arange(256, 256 + C, dtype=np.uint32)),
    ]
    keep = set(args.models.split(","))
    models = [m for m in models if m["name"] in keep]

    def signal():
        x = np.zeros((g.n, C), dtype=np.float32)
        x[src, np.arange(C)] = 1.0
        return x

    cfg = {"workload": "+".join(m["name"] for m in models) + f", {C} sources each, rmat scale 22",
           "graph": g.describe(), "lambda_1": lam, "columns_per_call": C,
           "models": {m["name"]: {"a": m["a"], "b": m["b"], "L": len(m["w"]) - 1, "eps": m["eps"]}
                      for m in models}}
    return host_workload(g, signal, models, cfg, "queries")


def workload_gnn_hkpr(args):
    from paper_2106_03058_amd import inputs

    def make():
        return inputs.chung_lu(2_400_000, 50, 2.5, seed=3, self_loops=True), {}

    g, _ = cached(args.cache, "chunglu_2m4_d50_s3_loops", make)
    C = min(args.columns, 128)
    models = [dict(name="hkpr", a=0.5, b=0.5, w=inputs.weights_hkpr(5.0, 10), eps=1e-7,
                   qids=np.arange(C, dtype=np.uint32))]

    def signal():
        return np.ascontiguousarray(inputs.features_normal(g.n, 128, seed=303)[:, :C])

    cfg = {"workload": f"gnn heat-kernel feature propagation, {C} N(0,1) columns, chung-lu n=2.4M d=50",
           "graph": g.describe(), "columns_per_call": C,
           "models": {"hkpr": {"a": 0.5, "b": 0.5, "L": 10, "t": 5.0, "eps": 1e-7}}}
    return host_workload(g, signal, models, cfg, "columns")


def workload_directed(args):
    """Directed proximity on R-MAT scale 22 (16 arcs per node, arcs kept as
    generated): PPR from 256 sources along out-edges (A~ = A^T) and
    single-target PPR to 256 targets along in-edges (A~ = A)."""
    import torch

    from paper_2106_03058_amd import agp, inputs

    g, _ = cached(args.cache, "rmat22_ef16_s2_directed",
                  lambda: (inputs.rmat(22, 16, 0.57, 0.19, 0.19, seed=2, directed=True), {}))
    C = min(args.columns, 256)
    outdeg = np.diff(g.row_ptr)
    indeg = np.bincount(g.col, minlength=g.n)
    rng = np.random.default_rng(102)
    src = rng.choice(np.flatnonzero(outdeg >= 1), size=C, replace=False)
    tgt = rng.choice(np.flatnonzero(indeg >= 1), size=C, replace=False)
    models = [
        dict(name="ppr", a=0.0, b=1.0, w=inputs.weights_ppr(0.2, 20), eps=1e-7,
             qids=np.arange(C, dtype=np.uint32), reverse=False, units=src),
        dict(name="single_target", a=1.0, b=0.0, w=inputs.weights_ppr(0.2, 20), eps=1e-7,
             qids=np.arange(256, 256 + C, dtype=np.uint32), reverse=True, units=tgt),
    ]
    keep = set(args.models.split(","))
    if not keep & {"ppr", "single_target"}:
        keep = {"ppr", "single_target"}
    models = [m for m in models if m["name"] in keep]
    state = {}

    def make_graph():
        # one handle per direction; each model uses its own
        state["G"] = {r: agp.Graph.from_inputs(g, directed=True, reverse=r) for r in {m["reverse"] for m in models}}
        return state["G"][models[0]["reverse"]]

    def signal_device():
        # one-hot columns: sources for the forward model, targets for the reverse one
        state["x"] = {}
        state["dx"] = {}
        for r, units in ((False, src), (True, tgt)):
            x = np.zeros((g.n, C), dtype=np.float32)
            x[units, np.arange(C)] = 1.0
            state["x"][r] = x
            state["dx"][r] = torch.from_numpy(x).to("cuda:0")
        return state["dx"][models[0]["reverse"]]

    def oracle_inputs(cols):
        return g, {r: np.ascontiguousarray(state["x"][r][:, cols]) for r in (False, True)}

    def oracle_graph_of(gh, m):
        import oracle

        return oracle.directed(gh, m["reverse"])

    def exact_of(gh, m, x):
        from oracle import dense

        return (dense.horner_sparse_directed(gh, m["a"], m["b"], m["w"], x, m["reverse"]),
                np.diff(gh.row_ptr))  # MaxError of a directed graph divides by out-degrees

    cfg = {"workload": "directed " + "+".join(m["name"] for m in models) + f", {C} sources/targets each, "
                       "rmat scale 22 (arcs as generated)",
           "graph": g.describe(), "columns_per_call": C,
           "models": {m["name"]: {"a": m["a"], "b": m["b"], "L": len(m["w"]) - 1, "eps": m["eps"],
                                  "pushes_along": "in-edges" if m["reverse"] else "out-edges"} for m in models}}
    return dict(n=g.n, make_graph=make_graph, signal_device=signal_device, models=models, cfg=cfg,
                unit="queries", oracle_inputs=oracle_inputs, state=state,
                graph_of=lambda m: state["G"][m["reverse"]], signal_of=lambda m: state["dx"][m["reverse"]],
                oracle_graph_of=oracle_graph_of, oracle_signal_of=lambda xh, m: xh[m["reverse"]],
                exact_of=exact_of)


def workload_gnn_ppr_large(args):
    """PPR (APPNP) feature propagation at the scale of a 111M-node citation
    graph: Chung-Lu, exponent 2.2, ~1.6e9 arcs plus a loop per node, generated
    on the GPU; an n x 128 U[-1, 1] feature matrix resident in HBM."""
    import torch

    from paper_2106_03058_amd import agp, inputs

    n = args.large_n
    arcs = int(round(1_615_685_872 * n / 111_059_956))
    state = {}

    def make_graph():
        t = time.time()
        _, rp, col = inputs.chung_lu_device(n, arcs / n, 2.2, seed=5, target_edges=arcs // 2)
        state["desc"] = {"n": n, "arcs_without_loops": int(rp[-1].item()),
                         "max_degree_without_loops": int((rp[1:] - rp[:-1]).max().item())}
        log(f"chung-lu n={n}: {state['desc']} in {time.time() - t:.1f}s")
        if args.host_leg:  # the same graph with its loops, for the oracle and the exact sums
            t = time.time()
            rpl, coll = inputs.add_self_loops_device(n, rp, col)
            state["host"] = inputs.Graph(n, rpl.cpu().numpy(), coll.cpu().numpy())
            del rpl, coll
            log(f"host copy of the graph with loops {time.time() - t:.1f}s")
        G = agp.Graph(rp, col, self_loops=True)
        del rp, col
        torch.cuda.empty_cache()
        return G

    def signal_device():
        return inputs.features_uniform_device(n, 128, -1.0, 1.0, seed=505)

    def oracle_inputs(cols):
        return state["host"], np.ascontiguousarray(state["X"][:, torch.from_numpy(cols).to(state["X"].device)]
                                                   .cpu().numpy())

    models = [dict(name="ppr", a=0.5, b=0.5, w=inputs.weights_ppr(0.1, 10), eps=1e-8,
                   qids=np.arange(128, dtype=np.uint32))]
    cfg = {"workload": f"gnn ppr feature propagation, 128 U[-1,1] columns, chung-lu n={n} gamma=2.2 "
                       f"(~{arcs:.3g} arcs + loops), resident in HBM",
           "graph": state, "columns_per_call": 128,
           "models": {"ppr": {"a": 0.5, "b": 0.5, "L": 10, "alpha": 0.1, "eps": 1e-8}}}
    return dict(n=n, make_graph=make_graph, signal_device=signal_device, models=models, cfg=cfg, unit="columns",
                oracle_inputs=oracle_inputs, state=state, cpu_sample=dict(stop_level=0, stride=8, units=4),
                single=2)


WORKLOADS = {"katz-tp": workload_katz_tp, "gnn-hkpr": workload_gnn_hkpr, "gnn-ppr-large": workload_gnn_ppr_large,
             "directed": workload_directed}


def run_serve(args) -> dict:
    """Served query stream: Poisson arrivals of single-source queries (1/3
    PPR with alpha ~ U[0.1, 0.3], 1/3 Katz, 1/3 transition probability;
    L ~ U{10..40}; eps ~ U{1e-5, 1e-6, 1e-7}; sources drawn proportional to
    degree) on an R-MAT scale-24 graph (32 edges per node), admitted into the
    continuous-batching server, against the same queries one per launch."""
    import torch

    from paper_2106_03058_amd import agp, inputs

    dev = torch.device("cuda:0")
    t = time.time()
    n, rp, col = inputs.rmat_device(24, 32, 0.57, 0.19, 0.19, seed=4, device=dev)
    nnz = int(rp[-1].item())
    log(f"rmat24: n={n} arcs={nnz} in {time.time() - t:.1f}s")
    t = time.time()
    lam = inputs.lambda_max_device(n, rp, col, tol=1e-10, max_iter=1000)
    log(f"lambda_1 = {lam:.6f} in {time.time() - t:.1f}s")
    G = agp.Graph(rp, col)
    deg = (rp[1:] - rp[:-1]).cpu().numpy().astype(np.float64)
    host = inputs.Graph(n, rp.cpu().numpy(), col.cpu().numpy()) if args.oracle_queries > 0 else None
    del rp, col
    torch.cuda.empty_cache()
    rng = np.random.default_rng(404)
    N = args.queries
    src = rng.choice(n, size=N, p=deg / deg.sum())
    qs = []
    for i in range(N):
        L = int(rng.integers(10, 41))
        eps = float(rng.choice([1e-5, 1e-6, 1e-7]))
        kind = i % 3
        if kind == 0:
            qs.append(("ppr", 0.0, 1.0, inputs.weights_ppr(float(rng.uniform(0.1, 0.3)), L), eps))
        elif kind == 1:
            qs.append(("katz", 0.0, 0.0, inputs.weights_katz(0.85 / lam, L, 0.85), eps))
        else:
            qs.append(("tp", 0.0, 1.0, inputs.weights_tp(L), eps))
    arrivals = np.cumsum(rng.exponential(1.0 / args.rate, size=N))
    S = args.slots
    pool = [torch.empty(n, dtype=torch.float32, device=dev) for _ in range(S + 32)]
    keep = min(args.single, N)
    kept = [torch.empty(n, dtype=torch.float32, device=dev) for _ in range(keep)]
    # queries re-run by the oracle keep their outputs in buffers of their own
    checked = sorted(np.random.default_rng(77).choice(N, size=min(args.oracle_queries, N), replace=False).tolist())
    held = {i: torch.empty(n, dtype=torch.float32, device=dev) for i in checked if i >= keep}
    srv = agp.Server(G, max_slots=S, queue_capacity=N + 1, memory_bytes=int(args.serve_memory_gb * 2**30))
    free = list(range(len(pool)))
    outstanding = {}
    lat, lat_admit, pushes, restarts = [], [], 0, 0
    submitted = 0
    t0 = time.perf_counter()
    while submitted < N or outstanding:
        now = time.perf_counter() - t0
        while submitted < N and arrivals[submitted] <= now and (submitted < keep or submitted in held or free):
            i = submitted
            name, a, b, w, eps = qs[i]
            slot = -1 if (i < keep or i in held) else free.pop()
            buf = kept[i] if i < keep else (held[i] if i in held else pool[slot])
            tk = srv.submit(int(src[i]), a, b, w, eps, 5000 + i, i, buf)
            outstanding[tk] = (i, slot)
            submitted += 1
        done = []
        for tk, (i, slot) in outstanding.items():
            r = srv.poll(tk)
            if r is not None:
                t_done = time.perf_counter() - t0
                lat.append((t_done - arrivals[i]) * 1e3)
                lat_admit.append(r["end_ms"] - r["submit_ms"])
                pushes += r["pushes"]
                restarts += r["restarts"]
                done.append(tk)
                if len(lat) % 128 == 0:
                    log(f"served {len(lat)}/{N} ({time.perf_counter() - t0:.1f}s)")
                if slot >= 0:
                    free.append(slot)
        for tk in done:
            del outstanding[tk]
        if not done:
            time.sleep(0.0002)
    makespan = time.perf_counter() - t0 - arrivals[0]
    srv.close()
    lat = np.array(lat)
    # the same first queries, one per launch (identical results by construction)
    lat1, pushes1, same = [], 0, True
    for i in range(keep):
        name, a, b, w, eps = qs[i]
        x = torch.zeros((n, 1), dtype=torch.float32, device=dev)
        x[int(src[i]), 0] = 1.0
        torch.cuda.synchronize()
        ts = time.perf_counter()
        o, st = agp.propagate(G, a, b, w, x, eps, 5000 + i, qids=[i], stats=True)
        lat1.append((time.perf_counter() - ts) * 1e3)
        pushes1 += st["pushes"]
        same &= bool(torch.equal(o[:, 0], kept[i]))
    lat1 = np.array(lat1)
    oracle_check = None
    if checked:
        import oracle
        from concurrent.futures import ThreadPoolExecutor

        t = time.time()
        sg = oracle.degree_sort(host)
        log(f"oracle degree sort {time.time() - t:.1f}s")
        t = time.time()
        ok = []

        def one(i):
            name, a, b, w, eps = qs[i]
            x = np.zeros(n, dtype=np.float32)
            x[int(src[i])] = 1.0
            ref, _ = oracle.propagate(sg, a, b, w, x, eps, 5000 + i, qids=[i], threads=1)
            got = (kept[i] if i < keep else held[i]).cpu().numpy().astype(np.float64)
            return i, bool(np.array_equal(got, ref))

        workers = min(16, os.cpu_count() or 1)
        with ThreadPoolExecutor(max_workers=workers) as ex:
            for k, (i, eq) in enumerate(ex.map(one, checked)):
                ok.append(eq)
                if k % 10 == 0 or not eq:
                    log(f"oracle query {k + 1}/{len(checked)} (#{i}): {'equal' if eq else 'DIFFERENT'}")
        oracle_check = {"queries": len(checked), "bit_exact": int(sum(ok)), "threads": workers,
                        "seconds": time.time() - t}
        log(f"oracle check {oracle_check}")
    return {
        "metric": METRIC,
        "value": pushes / makespan,
        "unit": "edge-pushes/s",
        "n_gpus": 1,
        "steps": 1,
        "warmup": 0,
        "ms_per_step": makespan * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"served stream of {N} queries (ppr/katz/tp, L 10-40, eps 1e-5..1e-7) "
                               f"at {args.rate:g}/s offered, rmat scale 24",
                   "graph": {"n": n, "arcs": nnz}, "lambda_1": lam, "slots": S,
                   "table_memory_gb": args.serve_memory_gb or "a quarter of the free memory"},
        "table_restarts": restarts,
        "queries_per_s_served": N / makespan,
        "latency_ms_served": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                              "note": "arrival to completion, including queueing"},
        "queries_per_s_one_per_launch": 1e3 / lat1.mean(),
        "latency_ms_one_per_launch": {"p50": float(np.percentile(lat1, 50)),
                                      "p99": float(np.percentile(lat1, 99)), "queries": keep},
        "pushes_per_s_one_per_launch": pushes1 / (lat1.sum() / 1e3),
        "served_equals_one_per_launch": same,
        "oracle_check": oracle_check,
    }


def run_cluster(args) -> dict:
    """Local clustering (Section 5): heat kernel PageRank (t = 5, a = 0,
    b = 1, L = 20, eps = 1e-7) from 64 seed nodes in one call, then the
    minimum-conductance sweeps of the 64 columns in one batched call, on an
    Orkut-shaped Chung-Lu graph (3,072,441 nodes, 117,185,083 edges,
    exponent 2.3) generated on the GPU.  One step = the propagation plus the
    64 sweeps."""
    import torch

    from paper_2106_03058_amd import agp, inputs

    dev = torch.device("cuda:0")
    n, edges = 3_072_441, 117_185_083
    t = time.time()
    _, rp, col = inputs.chung_lu_device(n, 2.0 * edges / n, 2.3, seed=6, target_edges=edges, device=dev)
    nnz = int(rp[-1].item())
    log(f"chung-lu n={n}: {nnz} arcs in {time.time() - t:.1f}s")
    deg = (rp[1:] - rp[:-1]).cpu().numpy()
    host = None if args.no_cpu_baseline else inputs.Graph(n, rp.cpu().numpy(), col.cpu().numpy())
    G = agp.Graph(rp, col)
    del rp, col
    torch.cuda.empty_cache()
    C = min(args.columns, 64)
    seeds = np.random.default_rng(606).choice(np.flatnonzero(deg >= 1), size=C, replace=False)
    X = torch.zeros((n, C), dtype=torch.float32, device=dev)
    X[torch.from_numpy(seeds).to(dev), torch.arange(C, device=dev)] = 1.0
    a, b, w, eps = 0.0, 1.0, inputs.weights_hkpr(5.0, 20), 1e-7
    qids = np.arange(C, dtype=np.uint32)
    out = torch.empty_like(X)

    def step():
        t0 = time.perf_counter()
        _, st = agp.propagate(G, a, b, w, X, eps, args.seed, qids=qids, out=out, stats=True)
        t1 = time.perf_counter()
        sizes, phis = agp.sweep_batch(G, out)
        t2 = time.perf_counter()
        return st, list(zip(sizes.tolist(), phis.tolist())), (t1 - t0) * 1e3, (t2 - t1) * 1e3

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    runs = [step() for _ in range(args.steps)]
    torch.cuda.synchronize()
    ms_per_step = (time.perf_counter() - t0) * 1e3 / args.steps
    st, clusters, _, _ = runs[0]
    for r in runs[1:]:
        assert r[1] == clusters
    prop_ms = float(np.mean([r[2] for r in runs]))
    sweep_ms = float(np.mean([r[3] for r in runs])) / C
    # the batched sweeps against one sweep per call (same results)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    single = [agp.sweep(G, out[:, c], order=False)[:2] for c in range(8)]
    torch.cuda.synchronize()
    single_ms = (time.perf_counter() - t1) * 1e3 / 8
    assert single == clusters[:8]
    # algorithmic bytes of one sweep: per arc the neighbour id and its rank
    # (8 B); per node the estimate and degree (8 B), keys and ids written and
    # read back by the radix sort (8 passes of 12 B each way), the rank
    # scatter (8 B), the row bounds (16 B), the two differences written and
    # scanned (16 + 32 B) and read for Phi (16 B)
    sweep_bytes = 8.0 * nnz + n * (8 + 12 + 8 * 24 + 8 + 16 + 48 + 16)
    sweep_gbps = sweep_bytes / (sweep_ms / 1e3) / 1e9
    sizes = np.array([c[0] for c in clusters])
    phis = np.array([c[1] for c in clusters])
    log(f"{ms_per_step:.1f} ms/step: propagation {prop_ms:.1f} ms, sweep {sweep_ms:.2f} ms each batched "
        f"({single_ms:.2f} ms one per call); "
        f"cluster sizes median {int(np.median(sizes))}, conductance median {np.median(phis):.4f}")
    result = {
        "metric": "local clusters/s (HKPR estimate + minimum-conductance sweep)",
        "value": C / (ms_per_step / 1e3),
        "unit": "clusters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"local clustering: hkpr t=5 L=20 eps=1e-7 from {C} seeds + sweep, "
                               "orkut-shaped chung-lu n=3.07M",
                   "graph": {"n": n, "arcs": nnz}, "seeds": C},
        "propagation_ms": prop_ms,
        "pushes_per_step": int(st["pushes"]),
        "edge_pushes_per_s_propagation": st["pushes"] / (prop_ms / 1e3),
        "sweep_ms_each": sweep_ms,
        "sweep_ms_one_per_call": single_ms,
        "sweep_roofline": {"bound": "hbm", "achieved": sweep_gbps, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                           "frac": sweep_gbps / HBM_PEAK_GBPS, "alg_bytes_per_sweep": sweep_bytes,
                           "note": "agp_sweep_batch of the step's 64 columns (all kernels and host waits), "
                                   "per column, against a single sweep's algorithmic bytes"},
        "cluster_size": {"median": int(np.median(sizes)), "min": int(sizes.min()), "max": int(sizes.max())},
        "conductance": {"median": float(np.median(phis)), "min": float(phis.min()), "max": float(phis.max())},
    }
    if host is not None:
        import oracle

        c = int(np.random.default_rng(55).integers(C))
        t = time.time()
        sg = oracle.degree_sort(host)
        t_sort = time.time() - t
        t = time.time()
        ref, cnt = oracle.propagate(sg, a, b, w, inputs.one_hot(n, [seeds[c]]), eps, args.seed,
                                    qids=qids[c:c + 1], wp=32)
        t_prop = time.time() - t
        t = time.time()
        rs, rphi, rorder = oracle.sweep(host, ref[:, 0])
        t_sw = time.time() - t
        gs, gphi, gorder = agp.sweep(G, out[:, c])
        same = bool(np.array_equal(out[:, c].cpu().numpy().astype(np.float64), ref[:, 0]))
        same &= (gs, gphi) == (rs, rphi) and bool(np.array_equal(gorder.cpu().numpy(), rorder))
        log(f"oracle: sort {t_sort:.1f}s, propagation {t_prop:.1f}s, sweep {t_sw:.2f}s; parity {same}")
        result["cpu_baseline"] = {"value": 1.0 / (t_prop + t_sw), "unit": "clusters/s", "cores": 1,
                                  "kind": "oracle",
                                  "sample": f"seed column {c}: oracle propagation {t_prop:.1f}s + sweep "
                                            f"{t_sw:.2f}s on one thread (degree sort {t_sort:.1f}s not counted)"}
        result["parity_full_size"] = {"columns": [c], "estimate_bit_exact_and_same_cluster": same,
                                      "cluster_size": int(rs), "conductance": float(rphi)}
    return result


def run_variants(args) -> dict:
    """The paper-literal variants against the defaults, each at the same eps,
    on a Chung-Lu graph generated on the GPU (n = 2.4M, mean degree 50,
    exponent 2.5, one loop per node):
      * signed features (GNN heat kernel, a = b = 1/2, t = 5, L = 10,
        eps = 1e-7, 32 N(0,1) columns): one signed pass against x+ and x-
        propagated separately;
      * PPR (alpha = 0.2, L = 20, a = 0, b = 1, eps = 1e-7) from 64 sources:
        truncated Y_i against the infinite-tail Y_i.
    Reported per case: time and edge pushes per call, and the error against
    the exact FP64 sum of Eq. 1 on two columns (sparse Horner on the host)."""
    import torch

    from oracle import dense
    from paper_2106_03058_amd import agp, inputs

    dev = torch.device("cuda:0")
    n = 2_400_000
    t = time.time()
    _, rp, col = inputs.chung_lu_device(n, 50.0, 2.5, seed=3, target_edges=n * 25, device=dev)
    host = inputs.add_self_loops(n, rp.cpu().numpy(), col.cpu().numpy())
    G = agp.Graph(rp, col, self_loops=True)
    deg = (rp[1:] - rp[:-1]).cpu().numpy()
    del rp, col
    torch.cuda.empty_cache()
    log(f"chung-lu n={n} with loops: {G.nnz} arcs in {time.time() - t:.1f}s")
    gen = torch.Generator(device=dev)
    gen.manual_seed(303)
    Xf = torch.randn((n, 32), generator=gen, device=dev, dtype=torch.float32)
    src = np.random.default_rng(102).choice(np.flatnonzero(deg >= 1), size=64, replace=False)
    Xs = torch.zeros((n, 64), dtype=torch.float32, device=dev)
    Xs[torch.from_numpy(src).to(dev), torch.arange(64, device=dev)] = 1.0
    cases = [
        ("signed_one_pass", Xf, 0.5, 0.5, inputs.weights_hkpr(5.0, 10), {}),
        ("signed_split", Xf, 0.5, 0.5, inputs.weights_hkpr(5.0, 10), {"split_signs": True}),
        ("ppr_truncated_Y", Xs, 0.0, 1.0, inputs.weights_ppr(0.2, 20), {}),
        ("ppr_infinite_tail", Xs, 0.0, 1.0, inputs.weights_ppr(0.2, 20), {"tail": True}),
    ]
    res = {}
    exact_cache = {}
    for name, X, a, b, w, kw in cases:
        out = torch.empty_like(X)
        for _ in range(args.warmup):
            agp.propagate(G, a, b, w, X, 1e-7, args.seed, out=out, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            _, st = agp.propagate(G, a, b, w, X, 1e-7, args.seed, out=out, stats=True, **kw)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / args.steps
        cols = [0, 1]
        got = out[:, cols].cpu().numpy().astype(np.float64)
        xh = X[:, cols].cpu().numpy().astype(np.float64)
        te = time.time()
        key = (id(X), a, b, len(w))
        if key not in exact_cache:  # both cases of a pair share the exact sum
            exact_cache[key] = dense.horner_sparse(host, a, b, w, xh)
        exact = exact_cache[key]
        diff = np.abs(got - exact)
        res[name] = {"ms_per_call": ms, "columns": X.shape[1], "edge_pushes": int(st["pushes"]),
                     "edge_pushes_per_s": st["pushes"] / (ms / 1e3),
                     "max_abs_err": float(diff.max()),
                     "rel_l1_err": float(diff.sum() / np.abs(exact).sum()),
                     "rel_l2_err": float(np.sqrt((diff ** 2).sum() / (exact ** 2).sum()))}
        log(f"{name}: {ms:.1f} ms, {st['pushes']:.3e} pushes, rel l1 {res[name]['rel_l1_err']:.3e} "
            f"(exact {time.time() - te:.1f}s)")
    # full-size parity of one sampled column of each variant against the oracle
    import oracle

    t = time.time()
    sg = oracle.degree_sort(host)
    parity = {}
    for name, X, a, b, w, kw in cases:
        if not kw:
            continue
        c = int(np.random.default_rng(55).integers(X.shape[1]))
        out = torch.empty_like(X)
        agp.propagate(G, a, b, w, X, 1e-7, args.seed, out=out, **kw)
        xc = X[:, c].cpu().numpy().astype(np.float64)
        ref, _ = oracle.propagate(sg, a, b, w, xc, 1e-7, args.seed, qids=[c], **kw)
        parity[name] = {"column": c, "bit_exact": bool(np.array_equal(out[:, c].cpu().numpy().astype(np.float64), ref))}
    log(f"variant parity {parity} in {time.time() - t:.1f}s")
    base = res["signed_one_pass"]
    return {
        "metric": "edge-pushes/s (default one-pass signed propagation; variants alongside)",
        "value": base["edge_pushes_per_s"],
        "unit": "edge-pushes/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": base["ms_per_call"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "paper-literal variants vs defaults at eps=1e-7: split signs (gnn hkpr, 32 N(0,1) "
                               "columns) and infinite-tail Y_i (ppr from 64 sources), chung-lu n=2.4M d=50 + loops",
                   "graph": {"n": n, "arcs": G.nnz}},
        "cases": res,
        "parity_full_size": parity,
        "split_cost_ratio": res["signed_split"]["ms_per_call"] / base["ms_per_call"],
        "tail_cost_ratio": res["ppr_infinite_tail"]["ms_per_call"] / res["ppr_truncated_Y"]["ms_per_call"],
    }


def copy_probe_gbps(dev) -> float:
    """Device-to-device copy of 4 GiB (read + write bytes over the copy's
    HIP-event time): the HBM rate a plain streaming kernel reaches."""
    import torch

    src = torch.ones(1 << 30, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    best = 0.0
    for _ in range(5):
        e0.record()
        dst.copy_(src)
        e1.record()
        e1.synchronize()
        best = max(best, 2.0 * src.numel() * 4 / (e0.elapsed_time(e1) / 1e3) / 1e9)
    del src, dst
    torch.cuda.empty_cache()
    return best


def level_roofline(runs, models, args, C) -> dict:
    """Roofline object of the level kernel over the timed steps.

    The launches: frontier-list levels 1..L (the level kernel with the
    launches that make its deferred rows and suffixes), or node-major dense
    levels 0..L-1 (level L only converts residues); one launch per level and
    column tile.  Two floors bound a launch: its random draws (runs +
    candidates) at ALU_PEAK_GDRAWS, and its algorithmic bytes at the HBM
    peak.  `bound` is the one with the larger floor (the larger fraction);
    the other is reported beside it, with the measured HBM traffic while the
    kernel sources hash to the profiled ones."""
    dense = all(st["dense"] for r in runs for st, _ in r)
    draws = lvl_ms = alg = 0.0
    launches = 0
    for r in runs:
        for (st, _), m in zip(r, models):
            L = st["levels"]
            lv = range(0, L) if dense else range(1, L + 1)
            for i in lv:
                draws += float(st["runs"][i]) + float(st["cand"][i])
                lvl_ms += float(st["level_ms"][i])
            alg += alg_bytes(st, lv, m["a"] == 0.0)
            launches += len(lv) * max(int(st["tiles"]), 1)
    if lvl_ms <= 0.0:  # captured level loops are timed as a whole, not per level
        return None
    avg_s = lvl_ms / 1e3 / max(launches, 1)
    alg_gbps = alg / (lvl_ms / 1e3) / 1e9
    gdraws = draws / (lvl_ms / 1e3) / 1e9
    rec = TRAFFIC.get(args.workload)
    traffic = None
    if rec and rec["sources"] == kernel_sources_sha() and rec["columns"] == C and not args.tune and not dense:
        traffic = rec["bytes_per_launch"] / avg_s / 1e9
    kernel = ("k_dense_level (levels 0..L-1)" if dense else
              "k_level<float, false, false, G> + k_det_big<float, G> + k_samp_big<float, G> (levels 1..L; "
              "G = 2 record column groups on binned levels of tiles with n C >= 2^31, else 1)")
    alu = {"bound": "alu", "achieved": gdraws, "peak": ALU_PEAK_GDRAWS, "unit": "Gdraw/s",
           "frac": gdraws / ALU_PEAK_GDRAWS,
           "peak_derivation": f"{VALU_LANE_OPS:.4g} VALU lane-ops/s / {VALU_PER_DRAW} per draw",
           "draws_per_launch": draws / max(launches, 1)}
    hbm = {"bound": "hbm", "achieved": alg_gbps, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
           "frac": alg_gbps / HBM_PEAK_GBPS, "alg_bytes_per_launch": alg / max(launches, 1)}
    main_, other = (alu, hbm) if alu["frac"] >= hbm["frac"] else (hbm, alu)
    out = dict(main_)
    out.update({"kernel": kernel, "traffic": traffic, "traffic_unit": "GB/s",
                "traffic_bytes_per_launch": rec["bytes_per_launch"] if traffic is not None else None,
                "traffic_over_alg_bytes": (traffic / alg_gbps) if traffic else None,
                "avg_launch_ms": avg_s * 1e3, "launches": launches, "other_bound": other})
    return out


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--seed", type=int, default=2021)
    ap.add_argument("--workload", default="gnn-ppr-large",
                    choices=sorted(WORKLOADS) + ["serve", "cluster", "variants"])
    ap.add_argument("--queries", type=int, default=1024, help="serve: queries in the stream")
    ap.add_argument("--rate", type=float, default=2000.0, help="serve: offered arrivals per second")
    ap.add_argument("--slots", type=int, default=112, help="serve: server slots")
    ap.add_argument("--serve-memory-gb", type=float, default=0.0,
                    help="serve: device memory of the residue tables (0: a quarter of the free memory)")
    ap.add_argument("--single", type=int, default=None, help="units timed one per launch")
    ap.add_argument("--oracle-queries", type=int, default=0,
                    help="serve: queries of the stream re-run by the oracle (random sample)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tune", action="store_true",
                    help="autotune the execution choices per model before timing (default: library defaults)")
    ap.add_argument("--cpu-units", type=int, default=None, help="columns of the oracle timing sample")
    ap.add_argument("--cpu-stop-level", type=int, default=None,
                    help="oracle timing sample: stop after this level (-1: whole columns, checked bit for bit)")
    ap.add_argument("--cpu-stride", type=int, default=None,
                    help="oracle timing sample: at the stop level visit every k-th node only")
    ap.add_argument("--parity-columns", type=int, default=0,
                    help="columns re-run whole by the oracle and compared bit for bit (beside the timing sample)")
    ap.add_argument("--exact-units", type=int, default=4,
                    help="sampled units whose error against the exact FP64 sum is reported")
    ap.add_argument("--cache", default=os.environ.get("AGP_BENCH_CACHE", ""),
                    help="directory to keep the generated graph between runs")
    ap.add_argument("--models", default="katz,tp,hkpr", help="subset of the step to run (profiling)")
    ap.add_argument("--columns", type=int, default=256, help="columns per call (profiling)")
    ap.add_argument("--large-n", type=int, default=111_059_956, help="gnn-ppr-large: nodes")
    ap.add_argument("--no-copy-probe", action="store_true")
    ap.add_argument("--capture", action="store_true",
                    help="run every call's level loops as captured hipGraphs (tuning field capture)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="copy 1 GiB device to device first (reference for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        return 2
    args.host_leg = (not args.no_cpu_baseline) or args.exact_units > 0 or args.parity_columns > 0
    if args.capture:
        os.environ["AGP_CAPTURE"] = "1"

    import torch

    from paper_2106_03058_amd import agp

    agp.lib()
    dev = torch.device("cuda:0")
    if args.workload == "serve":
        args.single = 16 if args.single is None else args.single
        print(json.dumps(run_serve(args)), flush=True)
        return 0
    if args.workload == "cluster":
        print(json.dumps(run_cluster(args)), flush=True)
        return 0
    if args.workload == "variants":
        print(json.dumps(run_variants(args)), flush=True)
        return 0
    W = WORKLOADS[args.workload](args)
    models, cfg, unit_name, n = W["models"], W["cfg"], W["unit"], W["n"]
    samp = dict(stop_level=-1, stride=1, units=4)
    samp.update(W.get("cpu_sample", {}))
    if args.cpu_units is not None:
        samp["units"] = args.cpu_units
    if args.cpu_stop_level is not None:
        samp["stop_level"] = args.cpu_stop_level
    if args.cpu_stride is not None:
        samp["stride"] = args.cpu_stride
    single = args.single if args.single is not None else W.get("single", 16)
    copy_gbps = None
    if args.calibrate_copy:
        a_ = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        b_ = torch.empty_like(a_)
        b_.copy_(a_)
        torch.cuda.synchronize()
        del a_, b_
    elif not args.no_copy_probe:
        copy_gbps = copy_probe_gbps(dev)
        log(f"copy probe {copy_gbps:.0f} GB/s")
    t = time.time()
    G = W["make_graph"]()
    torch.cuda.synchronize()
    log(f"device graph build (degree sort) {time.time() - t:.2f}s, max degree {G.max_degree}")
    X = W["signal_device"]()
    if "state" in W:
        W["state"]["X"] = X
        if "desc" in W["state"]:
            cfg["graph"] = W["state"]["desc"]
    C = X.shape[1]
    # per model: its graph handle and signal (the same for most workloads)
    Gs = [W["graph_of"](m) if "graph_of" in W else G for m in models]
    Xs = [W["signal_of"](m) if "signal_of" in W else X for m in models]
    outs = [torch.empty_like(Xm) for Xm in Xs]

    tunings = {}
    if args.tune:
        for m, o, Gm, Xm in zip(models, outs, Gs, Xs):
            tunings[m["name"]] = agp.autotune(Gm, m["a"], m["b"], m["w"], Xm, m["eps"], args.seed,
                                              qids=m["qids"], out=o)
        log(f"autotuned: {tunings}")

    def step(stats: bool):
        res = []
        for m, o, Gm, Xm in zip(models, outs, Gs, Xs):
            t0 = time.perf_counter()
            _, st = agp.propagate(Gm, m["a"], m["b"], m["w"], Xm, m["eps"], args.seed, qids=m["qids"],
                                  out=o, stats=stats)
            res.append((st, (time.perf_counter() - t0) * 1e3))
        return res

    for k in range(args.warmup):
        step(True)
        log(f"warmup step {k + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    runs = []
    for k in range(args.steps):
        runs.append(step(True))
        log(f"step {k + 1}/{args.steps}: {sum(ms for _, ms in runs[-1]):.1f} ms")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    pushes_step = sum(st["pushes"] for st, _ in runs[0])
    for r in runs[1:]:  # identical seeds: identical work every step
        assert sum(st["pushes"] for st, _ in r) == pushes_step
    value = pushes_step / (ms_per_step / 1e3)
    log(f"{ms_per_step:.1f} ms/step, {pushes_step:.3e} pushes/step")

    roofline = level_roofline(runs, models, args, C)
    all_bytes = all_ms = 0.0
    for r in runs:
        for (st, _), m in zip(r, models):
            L = st["levels"]
            all_bytes += alg_bytes(st, range(L + 1), m["a"] == 0.0)
            all_ms += float(st["level_total_ms"].sum()) or float(st["device_ms"])
    per_level = []
    for (st, ms), m in zip(runs[0], models):
        per_level.append({"model": m["name"], "call_ms": round(ms, 3), "tiles": int(st["tiles"]),
                          "dense": bool(st["dense"]),
                          "frontier": [int(v) for v in st["frontier"]],
                          "pushes": [int(d + a) for d, a in zip(st["det"], st["acc"])],
                          "draws": [int(r_ + c_) for r_, c_ in zip(st["runs"], st["cand"])],
                          "level_ms": [round(float(v), 4) for v in st["level_ms"]],
                          "level_total_ms": [round(float(v), 4) for v in st["level_total_ms"]]})

    # batched vs one unit (query or column) per launch, same eps and keys
    lat_b = []
    for (st, ms), m in zip(runs[-1], models):
        lat_b += [ms] * C
    lat_b = np.array(lat_b)
    q_per_s_batched = len(models) * C / (ms_per_step / 1e3)
    lat_s = []
    nq = single // max(len(models), 1)
    # one input and one output buffer for every single-unit call (a captured
    # level loop is replayed when the buffers stay the same)
    one = torch.empty((n, 1), dtype=torch.float32, device=dev) if nq > 0 else None
    one_x = torch.empty((n, 1), dtype=torch.float32, device=dev) if nq > 0 else None
    single_ok = True
    for m, o, Gm, Xm in zip(models, outs, Gs, Xs):
        for c in range(min(nq, C)):
            one_x.copy_(Xm[:, c:c + 1])
            torch.cuda.synchronize()
            ts = time.perf_counter()
            agp.propagate(Gm, m["a"], m["b"], m["w"], one_x, m["eps"], args.seed, qids=m["qids"][c:c + 1], out=one)
            lat_s.append((time.perf_counter() - ts) * 1e3)
            single_ok &= bool(torch.equal(one[:, 0], o[:, c]))
    del one, one_x
    log(f"{len(lat_s)} units one per launch, equal to the batched columns: {single_ok}")

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
        "config": cfg,
        "tuning": tunings,
        "captured_level_loops": bool(args.capture),
        "pushes_per_step": pushes_step,
        "hbm_gbps_algorithmic_all_levels": all_bytes / (all_ms / 1e3) / 1e9,
        "hbm_copy_probe_gbps": copy_gbps,
        f"{unit_name}_per_s_batched": q_per_s_batched,
        "latency_ms_batched": {"p50": float(np.percentile(lat_b, 50)), "p99": float(np.percentile(lat_b, 99))},
        "roofline": roofline,
        "per_level": per_level,
    }
    if lat_s:
        lat_s = np.array(lat_s)
        result[f"{unit_name}_per_s_one_per_launch"] = 1e3 / lat_s.mean()
        result["latency_ms_one_per_launch"] = {"p50": float(np.percentile(lat_s, 50)),
                                               "p99": float(np.percentile(lat_s, 99)), "units": int(len(lat_s))}
        result["one_per_launch_equals_batched"] = single_ok
    print(json.dumps({"partial": True, "value": value, "ms_per_step": ms_per_step, "roofline": roofline}),
          file=sys.stderr, flush=True)

    if args.host_leg:
        host_leg(args, W, models, outs, C, samp, unit_name, result)
    print(json.dumps(result), flush=True)
    return 0


def host_leg(args, W, models, outs, C, samp, unit_name, result) -> None:
    """The oracle's timing sample, whole-column parity and the error against
    the exact FP64 sum, on sampled columns of the same inputs."""
    import torch

    import oracle

    dev = outs[0].device
    rng = np.random.default_rng(55)
    want = max(samp["units"] if not args.no_cpu_baseline else 0, args.exact_units, args.parity_columns)
    cols = np.sort(rng.choice(C, size=min(want, C), replace=False))
    gh, xh = W["oracle_inputs"](cols)
    xhs = [W["oracle_signal_of"](xh, m) if "oracle_signal_of" in W else xh for m in models]
    host_threads = min(16, os.cpu_count() or 1)
    got = [outs[mi][:, torch.from_numpy(cols).to(dev)].cpu().numpy().astype(np.float64)
           for mi in range(len(models))]
    if not args.no_cpu_baseline or args.parity_columns > 0:
        t = time.time()
        if "oracle_graph_of" in W:
            sgs = [W["oracle_graph_of"](gh, m) for m in models]
        else:
            sg = oracle.degree_sort(gh, threads=host_threads)
            sgs = [sg for _ in models]
        log(f"oracle degree sort {time.time() - t:.1f}s on {host_threads} threads")
    if not args.no_cpu_baseline:
        k = min(samp["units"], cols.size)
        threads = min(k * len(models), 16, os.cpu_count() or 1)
        results = {}

        def run(mi, m):
            results[mi] = oracle.propagate(sgs[mi], m["a"], m["b"], m["w"], xhs[mi][:, :k], m["eps"], args.seed,
                                           qids=m["qids"][cols[:k]], threads=max(threads // len(models), 1),
                                           stop_level=samp["stop_level"], sample_stride=samp["stride"])

        t = time.time()
        ths = [threading.Thread(target=run, args=(mi, m)) for mi, m in enumerate(models)]
        for th in ths:
            th.start()
        for th in ths:
            th.join()
        wall = time.time() - t
        tot_push = sum(int(results[mi][1]["det"].sum() + results[mi][1]["acc"].sum()) for mi in range(len(models)))
        whole = samp["stop_level"] < 0 and samp["stride"] == 1
        what = (f"{unit_name} {cols[:k].tolist()} of each model ({', '.join(m['name'] for m in models)})"
                + ("" if whole else f", level {samp['stop_level']} only"
                   + ("" if samp["stride"] == 1 else f", nodes with id % {samp['stride']} == 0")))
        result["cpu_baseline"] = {"value": tot_push / wall, "unit": "edge-pushes/s", "cores": threads,
                                  "kind": "oracle",
                                  "sample": f"{what}; same inputs and seeds; {tot_push} pushes in {wall:.1f}s "
                                            f"wall on {threads} threads (degree sort not counted)"}
        log(f"oracle sample {wall:.1f}s: {tot_push} pushes")
        if whole:
            parity = all(np.array_equal(got[mi][:, :k], results[mi][0]) for mi in range(len(models)))
            result["parity_full_size"] = {"units_checked": k * len(models), "columns": cols[:k].tolist(),
                                          "bit_exact": bool(parity)}
            log(f"parity of the sample: {parity}")
    if args.parity_columns > 0:
        k = min(args.parity_columns, cols.size)
        threads = min(k * len(models), 16, os.cpu_count() or 1)
        t = time.time()
        ok = True
        for mi, m in enumerate(models):
            ref, _ = oracle.propagate(sgs[mi], m["a"], m["b"], m["w"], xhs[mi][:, :k], m["eps"], args.seed,
                                      qids=m["qids"][cols[:k]], threads=threads)
            eq = np.array_equal(got[mi][:, :k], ref)
            log(f"parity {m['name']} columns {cols[:k].tolist()}: {'bit-exact' if eq else 'DIFFERENT'} "
                f"({time.time() - t:.0f}s)")
            ok &= bool(eq)
        result["parity_full_size"] = {"units_checked": k * len(models), "columns": cols[:k].tolist(),
                                      "bit_exact": ok, "oracle_seconds": time.time() - t, "threads": threads}
    if args.exact_units > 0:
        ke = min(args.exact_units, cols.size)
        t = time.time()
        errs = {}
        for mi, m in enumerate(models):
            if "exact_of" in W:
                exact, deg = W["exact_of"](gh, m, xhs[mi][:, :ke])
            else:
                exact = oracle.truncated_sum(gh, m["a"], m["b"], m["w"], xhs[mi][:, :ke], threads=host_threads,
                                             verbose=True)
                deg = np.diff(gh.row_ptr)
            diff = np.abs(got[mi][:, :ke] - exact)
            dn = np.maximum(deg, 1).astype(np.float64)[:, None]
            errs[m["name"]] = {
                "columns": cols[:ke].tolist(), "eps": m["eps"],
                "max_abs": [float(v) for v in diff.max(axis=0)],
                "max_abs_over_max_exact": [float(v) for v in diff.max(axis=0) / np.maximum(np.abs(exact).max(axis=0),
                                                                                             1e-300)],
                "rel_l1": [float(v) for v in diff.sum(axis=0) / np.maximum(np.abs(exact).sum(axis=0), 1e-300)],
                "max_error_degree_normalized": [float(v) for v in (diff / dn).max(axis=0)],
            }
        result["error_vs_exact"] = errs
        log(f"exact sums {time.time() - t:.1f}s: {errs}")


if __name__ == "__main__":
    sys.exit(main())
