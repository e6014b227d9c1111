"""Dense levels (node-major, one lane per column) against the oracle.

Feature propagation has dense frontiers (every feature of level 0 is
non-zero), so the library runs such calls node by node with one lane per
signal column instead of through (node, column) frontier lists.  The random
decisions and the exact sums are those of Algorithm 2 under the same
specification, so estimates and every per-level counter must equal the
oracle's bit for bit: on graphs with self-loops (the GNN convention),
isolated nodes and rows long enough to be cut into pieces, for signed and
non-negative signals, a = 0 and a > 0, column tiles with a ragged tail,
several record groups, record buffers that overflow, and atomics only.
"""
import numpy as np
import pytest

import oracle
from paper_2106_03058_amd import inputs

pytestmark = pytest.mark.gpu

HUBS = (4200, 9000)  # rows above the 4096 arcs that cut a row into pieces


def _graph(n=12000, loops=True, hubs=True, seed=21):
    g = inputs.chung_lu(n, 10, 2.3, seed=seed, self_loops=False)
    if not hubs:
        if loops:
            rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
            return inputs.csr_from_pairs(g.n, rows, g.col.astype(np.int64), self_loops=True)
        return g
    rng = np.random.default_rng(seed)
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    src, dst = [rows], [g.col.astype(np.int64)]
    for h, d in enumerate(HUBS):
        nb = rng.choice(np.arange(len(HUBS), n), size=d, replace=False)
        src.append(np.full(d, n - 1 - h))  # hubs at the end of the id range
        dst.append(nb)
    return inputs.csr_from_pairs(n, np.concatenate(src), np.concatenate(dst), self_loops=loops)


@pytest.fixture(scope="module")
def env():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2106_03058_amd import agp

    agp.lib()
    g = _graph()
    deg = np.diff(g.row_ptr)
    assert deg.max() > 4096 and (deg > 4096).sum() == len(HUBS)
    return torch, agp, g, agp.Graph.from_inputs(g, validate=True), oracle.degree_sort(g)


def _signal(n, C, kind, seed=5):
    if kind == "normal":
        return inputs.features_normal(n, C, seed=seed)
    if kind == "uniform":
        return inputs.features_uniform(n, C, 0.0, 1.0, seed=seed)
    if kind == "sparse":  # dense enough for the dense path, with zero entries and a zero column
        x = inputs.features_normal(n, C, seed=seed)
        x[np.random.default_rng(seed).random((n, C)) < 0.5] = 0.0
        x[:, 0] = 0.0
        return x
    raise ValueError(kind)


MODELS = {
    # name: (a, b, weights, eps, signal)
    "gnn_hkpr": (0.5, 0.5, inputs.weights_hkpr(5.0, 10), 3e-5, "normal"),
    "gnn_ppr_fine": (0.5, 0.5, inputs.weights_ppr(0.1, 10), 2e-6, "normal"),
    "appnp_uniform": (0.0, 1.0, inputs.weights_ppr(0.2, 8), 1e-5, "uniform"),
    "general_ab": (0.3, 0.7, inputs.weights_hkpr(3.0, 6), 1e-5, "normal"),
    "katz": (0.0, 0.0, inputs.weights_katz(0.02, 6, 0.85), 1e-5, "uniform"),
    "tp": (0.0, 1.0, inputs.weights_tp(5), 1e-5, "sparse"),
    "single_target": (1.0, 0.0, inputs.weights_ppr(0.2, 6), 1e-5, "uniform"),
}


def _check(torch, agp, G, sg, a, b, w, x, eps, seed, monkeypatch, *, env_vars=None, qids=None):
    monkeypatch.setenv("AGP_DENSE", "1")
    for k, v in (env_vars or {}).items():
        monkeypatch.setenv(k, v)
    X = torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")
    out, st = agp.propagate(G, a, b, w, X, eps, seed, qids=qids, stats=True)
    got = out.cpu().numpy().astype(np.float64)
    ref, cnt = oracle.propagate(sg, a, b, w, x, eps, seed, qids=qids, threads=8)
    L = len(w) - 1
    bad = ~np.isclose(got, ref, rtol=1e-5, atol=1e-9)
    assert not bad.any(), f"{bad.sum()} entries outside tolerance, max diff {np.abs(got - ref).max()}"
    assert np.array_equal(got, ref), f"not bit-identical: max diff {np.abs(got - ref).max()}"
    for k in ("frontier", "hash", "det", "cand", "acc", "runs"):
        want = cnt[k].sum(axis=0).astype(np.uint64)
        assert np.array_equal(st[k][: L + 1], want[: L + 1]), f"counter {k}: {st[k][:L + 1]} vs {want}"
    return got, st


@pytest.mark.parametrize("name", sorted(MODELS))
@pytest.mark.parametrize("C", [5, 64, 70])
def test_dense_levels_equal_oracle(env, monkeypatch, name, C):
    torch, agp, g, G, sg = env
    a, b, w, eps, kind = MODELS[name]
    x = _signal(g.n, C, kind)
    print(f"dense {name} C={C}", flush=True)
    _, st = _check(torch, agp, G, sg, a, b, w, x, eps, 2024, monkeypatch)
    assert st["pushes"] > 0


@pytest.mark.parametrize("C,env_vars", [
    (70, {"AGP_AGGREGATION": "atomic"}),
    (70, {"AGP_RECORD_CAP": "3000"}),                               # records overflow the buffers
    (70, {"AGP_DENSE_GROUP_SHIFT": "4"}),                           # tiles of 35: groups of 16, 16, 3
    (64, {"AGP_DENSE_GROUP_SHIFT": "3", "AGP_COLUMN_TILE": "32"}),  # tiles of 32: 4 groups of 8
    (70, {"AGP_COLUMN_TILE": "7"}),                                 # 10 tiles of 7
    (70, {"AGP_COLUMN_TILE": "30"}),                                # 3 tiles of 24 (ragged last: 22)
])
def test_dense_execution_choices_keep_the_bits(env, monkeypatch, C, env_vars):
    torch, agp, g, G, sg = env
    a, b, w, eps, kind = MODELS["gnn_hkpr"]
    x = _signal(g.n, C, kind, seed=9)
    print(f"dense choices {env_vars}", flush=True)
    _check(torch, agp, G, sg, a, b, w, x, eps, 77, monkeypatch, env_vars=env_vars)


def test_dense_equals_frontier_lists(env, monkeypatch):
    """The dense path and the frontier-list path give the same bits (and the
    automatic choice takes the dense path for a dense signal)."""
    torch, agp, g, G, sg = env
    a, b, w, eps, _ = MODELS["gnn_ppr_fine"]
    X = torch.from_numpy(_signal(g.n, 40, "normal", seed=3)).to("cuda:0")
    monkeypatch.setenv("AGP_DENSE", "0")
    o1, s1 = agp.propagate(G, a, b, w, X, eps, 5, stats=True)
    monkeypatch.setenv("AGP_DENSE", "auto")
    o2, s2 = agp.propagate(G, a, b, w, X, eps, 5, stats=True)
    assert torch.equal(o1, o2)
    for k in ("frontier", "hash", "det", "cand", "acc", "runs"):
        assert np.array_equal(s1[k], s2[k])


def test_dense_qids_and_level_counts(env, monkeypatch):
    torch, agp, g, G, sg = env
    a, b, _, eps, kind = MODELS["gnn_hkpr"]
    x = _signal(g.n, 9, kind, seed=4)
    qids = np.array([7, 1000, 3, 99999, 5, 6, 123456, 8, 2], dtype=np.uint32)
    for L in (0, 1, 2):
        w = inputs.weights_hkpr(5.0, L)
        print(f"dense L={L}", flush=True)
        _check(torch, agp, G, sg, a, b, w, x, eps, 11, monkeypatch, qids=qids)


@pytest.mark.parametrize("loops", [False, True])
def test_dense_without_long_rows_and_isolated_nodes(env, monkeypatch, loops):
    torch, agp, *_ = env
    g = _graph(n=6000, loops=loops, hubs=False, seed=8)
    if not loops:
        assert (np.diff(g.row_ptr) == 0).any()  # isolated nodes
    G = agp.Graph.from_inputs(g, validate=True)
    sg = oracle.degree_sort(g)
    a, b, w, eps, kind = MODELS["gnn_hkpr"]
    _check(torch, agp, G, sg, a, b, w, _signal(g.n, 33, kind, seed=1), eps, 3, monkeypatch)


def test_dense_out_of_range_is_reported_and_recovers(env, monkeypatch):
    """A threshold so small that the exact sums could wrap: AGP_ERANGE, and
    the next call (residues and sums restored to zero) is exact again."""
    torch, agp, g, G, sg = env
    a, b, w, _, kind = MODELS["gnn_hkpr"]
    x = _signal(g.n, 8, kind, seed=2)
    monkeypatch.setenv("AGP_DENSE", "1")
    X = torch.from_numpy(x).to("cuda:0")
    with pytest.raises(agp.AGPError) as e:
        agp.propagate(G, a, b, w, X, 1e-20, 1)
    assert e.value.code == agp.AGP_ERANGE
    x2 = _signal(g.n, 8, kind, seed=6)
    _check(torch, agp, G, sg, a, b, w, x2, 3e-5, 4, monkeypatch)


def test_dense_calls_with_changing_layouts(env, monkeypatch):
    """Consecutive calls whose record groups and bin counts differ reuse the
    same scratch memory: each call still starts from cleared counters."""
    torch, agp, g, G, sg = env
    a, b, w, eps, kind = MODELS["gnn_hkpr"]
    seq = [(64, {"AGP_DENSE_GROUP_SHIFT": "3", "AGP_COLUMN_TILE": "32"}),
           (70, {"AGP_COLUMN_TILE": "7"}),
           (40, {"AGP_DENSE_GROUP_SHIFT": "2"}),
           (70, {})]
    for k, (C, env_vars) in enumerate(seq):
        for name in ("AGP_DENSE_GROUP_SHIFT", "AGP_COLUMN_TILE"):
            monkeypatch.delenv(name, raising=False)
        print(f"layout sequence step {k}: C={C} {env_vars}", flush=True)
        _check(torch, agp, G, sg, a, b, w, _signal(g.n, C, kind, seed=20 + k), eps, 5 + k, monkeypatch,
               env_vars=env_vars)
