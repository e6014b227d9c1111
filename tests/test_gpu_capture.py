"""The level loop captured into a hipGraph and replayed.

With the tuning field `capture`, a tile's level loop (every kernel from the
first level to the last compaction; the per-level values of a call sit in
device memory) is captured once per graph, column count, level count,
buffers and modes, and replayed by later calls.  Each replay must give the
oracle's bits and counters, and the same bits as a call launched kernel by
kernel, across seeds, signals rewritten in place, eager work between the
replays, new output buffers, binned levels and deferred rows.
"""
import numpy as np
import pytest

import oracle
from paper_2106_03058_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2106_03058_amd import agp

    agp.lib()
    g = inputs.chung_lu(9000, 12, 2.2, seed=23, self_loops=True)
    return torch, agp, g, agp.Graph.from_inputs(g, validate=True), oracle.degree_sort(g)


CASES = {
    # name: (a, b, weights, eps, signal, tuning besides capture)
    "ppr_onehot": (0.0, 1.0, inputs.weights_ppr(0.2, 10), 1e-6, "onehot", {}),
    "gnn_signed": (0.5, 0.5, inputs.weights_hkpr(4.0, 8), 2e-5, "normal", {}),
    "binned_deferred": (0.0, 1.0, inputs.weights_tp(6), 1e-6, "onehot", {"aggregation": 1, "big_row": 64,
                                                                          "big_items": 1}),
}


def _x(g, kind, C, seed):
    if kind == "onehot":
        return inputs.one_hot(g.n, inputs.sources_uniform(g, C, seed=seed))
    return inputs.features_normal(g.n, C, seed=seed)


def _check(agp, G, sg, a, b, w, X, xh, eps, seed, out):
    got, st = agp.propagate(G, a, b, w, X, eps, seed, out=out, stats=True)
    ref, cnt = oracle.propagate(sg, a, b, w, xh, eps, seed, threads=8)
    assert np.array_equal(got.cpu().numpy().astype(np.float64), ref)
    for k in ("frontier", "hash", "det", "cand", "acc", "runs"):
        assert np.array_equal(st[k], cnt[k].sum(axis=0).astype(np.uint64)), k
    return got, st


@pytest.mark.parametrize("name", sorted(CASES))
def test_replayed_level_loop_equals_oracle_and_direct_launches(env, name):
    torch, agp, g, G, sg = env
    a, b, w, eps, kind, extra = CASES[name]
    C = 16
    X = torch.empty((g.n, C), dtype=torch.float32, device="cuda:0")
    out = torch.empty_like(X)
    try:
        for k, seed in enumerate((5, 6, 7, 8)):
            xh = _x(g, kind, C, seed=10 + k)
            X.copy_(torch.from_numpy(xh))  # new signal, same buffer: the replay reads it
            torch.cuda.synchronize()
            agp.set_tuning(G, C, a, b, {**extra, "capture": 1})
            print(f"{name}: replay {k} seed {seed}", flush=True)
            got, st = _check(agp, G, sg, a, b, w, X, xh, eps, seed, out)
            assert st["device_ms"] > 0 and not st["level_ms"].any()  # timed as a whole
            kept = got.clone()
            torch.randn(1000, device="cuda:0").sum().item()  # eager work between replays
            agp.set_tuning(G, C, a, b, {**extra, "capture": 0})
            direct, _ = agp.propagate(G, a, b, w, X, eps, seed, out=torch.empty_like(X))
            assert torch.equal(direct, kept)
        # a new output buffer is a new capture
        agp.set_tuning(G, C, a, b, {**extra, "capture": 1})
        _check(agp, G, sg, a, b, w, X, xh, eps, 99, torch.empty_like(X))
    finally:
        agp.set_tuning(G, C, a, b, None)


def test_capture_with_other_level_counts_and_columns(env):
    torch, agp, g, G, sg = env
    a, b = 0.0, 1.0
    for L, C in ((0, 3), (1, 3), (12, 5), (12, 3)):
        w = inputs.weights_ppr(0.2, L)
        xh = _x(g, "onehot", C, seed=L)
        X = torch.from_numpy(xh).to("cuda:0")
        agp.set_tuning(G, C, a, b, {"capture": 1})
        try:
            for seed in (1, 2):
                print(f"L={L} C={C} seed {seed}", flush=True)
                _check(agp, G, sg, a, b, w, X, xh, 1e-6, seed, None)
        finally:
            agp.set_tuning(G, C, a, b, None)
