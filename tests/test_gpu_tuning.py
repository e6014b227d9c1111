"""Every execution choice the autotuner searches gives the oracle's bits.

The tuning (dense or frontier-list levels, aggregation, grid, column tile,
the cut-offs that defer long rows and large sampled suffixes, the sparse and
binned level cuts) changes only how a level is executed, never a random
decision or a sum: each candidate value is pinned with agp_set_tuning and
the estimate and counters compared with the oracle."""
import numpy as np
import pytest

import oracle
from paper_2106_03058_amd import inputs

pytestmark = pytest.mark.gpu

CANDIDATES = {
    "dense": [0, 1],
    "aggregation": [0, 1, 2],
    "level_blocks": [256, 1024, 8192],
    "tile_columns": [0, 7, 16],
    "big_row": [64, 1024, 16384],
    "big_items": [1, 16, 256],
    "sparse_shift": [1, 3, 9],
    "bin_shift": [1, 2, 6],
    "capture": [0, 1],
}


@pytest.fixture(scope="module")
def env():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2106_03058_amd import agp

    agp.lib()
    g = inputs.chung_lu(8000, 14, 2.2, seed=17, self_loops=True)
    return torch, agp, g, agp.Graph.from_inputs(g, validate=True), oracle.degree_sort(g)


WORKLOADS = {
    # one-hot proximity queries (frontier lists) and dense signed features
    "ppr_onehot": (0.0, 1.0, inputs.weights_ppr(0.2, 10), 1e-6, "onehot"),
    "gnn_signed": (0.5, 0.5, inputs.weights_hkpr(4.0, 8), 2e-5, "normal"),
}


def _x(g, kind):
    if kind == "onehot":
        return inputs.one_hot(g.n, inputs.sources_uniform(g, 24, seed=3))
    return inputs.features_normal(g.n, 24, seed=3)


@pytest.mark.parametrize("workload", sorted(WORKLOADS))
def test_every_tuning_candidate_keeps_the_bits(env, workload):
    torch, agp, g, G, sg = env
    a, b, w, eps, kind = WORKLOADS[workload]
    x = _x(g, kind)
    X = torch.from_numpy(x).to("cuda:0")
    C = x.shape[1]
    ref, cnt = oracle.propagate(sg, a, b, w, x, eps, 31, threads=8)
    try:
        for name, vals in CANDIDATES.items():
            for v in vals:
                print(f"{workload}: {name}={v}", flush=True)
                agp.set_tuning(G, C, a, b, {name: v})
                assert agp.get_tuning(G, C, a, b)[name] in (v, {0: "never", 1: "always", 2: "auto"}.get(v),
                                                            {0: "atomic", 1: "binned", 2: "auto"}.get(v))
                out, st = agp.propagate(G, a, b, w, X, eps, 31, stats=True)
                assert np.array_equal(out.cpu().numpy().astype(np.float64), ref), f"{name}={v}"
                for k in ("frontier", "hash", "det", "cand", "acc", "runs"):
                    assert np.array_equal(st[k], cnt[k].sum(axis=0).astype(np.uint64)), f"{name}={v}: {k}"
    finally:
        agp.set_tuning(G, C, a, b, None)


def test_autotune_pick_is_kept_and_normalized(env):
    torch, agp, g, G, sg = env
    a, b, w, eps, kind = WORKLOADS["gnn_signed"]
    x = _x(g, kind)[:, :20].copy()
    X = torch.from_numpy(x).to("cuda:0")
    pick = agp.autotune(G, a, b, w, X, eps, 8)
    assert agp.get_tuning(G, 20, a, b) == pick
    assert pick["big_row"] > 0 and pick["big_items"] > 0 and pick["sparse_shift"] > 0 and pick["bin_shift"] > 0
    ref, _ = oracle.propagate(sg, a, b, w, x, eps, 8, threads=8)
    out, _ = agp.propagate(G, a, b, w, X, eps, 8)
    assert np.array_equal(out.cpu().numpy().astype(np.float64), ref)
    agp.set_tuning(G, 20, a, b, None)
    assert agp.get_tuning(G, 20, a, b)["level_blocks"] == 4096
