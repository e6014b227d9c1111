"""Rows with thousands of deterministic pushes (hubs holding a large residue,
Algorithm 2's deterministic part of a push) are taken out of their wave and
pushed by the whole grid after the level; the estimates and counters stay
bit-exact with the oracle, in every aggregation mode and whatever the length
of the deferred list (AGP_BIG_ROWS: 0 turns the deferral off, 1 leaves all
but one row with their waves)."""
import numpy as np
import pytest

import oracle
from paper_2106_03058_amd import inputs

pytestmark = pytest.mark.gpu

HUBS = (4200, 6000, 9000, 12000)  # degrees of nodes 0..3: above the 4096 pushes that defer a row


def _hub_graph(n=16000, seed=7):
    rng = np.random.default_rng(seed)
    src = [rng.integers(0, n, size=5 * n)]
    dst = [rng.integers(0, n, size=5 * n)]
    for h, d in enumerate(HUBS):
        nb = rng.choice(np.arange(len(HUBS), n), size=d, replace=False)
        src.append(np.full(d, h))
        dst.append(nb)
    return inputs.csr_from_pairs(n, np.concatenate(src), np.concatenate(dst))


@pytest.fixture(scope="module")
def env():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2106_03058_amd import agp

    agp.lib()
    g = _hub_graph()
    deg = np.diff(g.row_ptr)
    assert all(deg[h] >= 4096 for h in range(len(HUBS)))
    return torch, agp, g, agp.Graph.from_inputs(g, validate=True), oracle.degree_sort(g)


def _onehot(g):
    return inputs.one_hot(g.n, [0, 1, 2, 3, 100, 2000])


CASES = {
    # name: (a, b, weights, eps, signal)
    "ppr": (0.0, 1.0, inputs.weights_ppr(0.2, 10), 1e-7, "onehot"),
    "katz": (0.0, 0.0, inputs.weights_katz(0.005, 8), 1e-7, "onehot"),
    "general_signed": (0.5, 0.5, inputs.weights_hkpr(3.0, 8), 1e-8, "normal"),
}


def _x(g, kind):
    if kind == "onehot":
        return _onehot(g)
    return inputs.features_normal(g.n, 3, seed=12)


def _check(got, st, ref, cnt, L):
    assert np.array_equal(got, ref), f"max diff {np.abs(got - ref).max()}"
    for k in ("frontier", "hash", "det", "cand", "acc", "runs"):
        assert np.array_equal(st[k][: L + 1], cnt[k].sum(axis=0).astype(np.uint64)[: L + 1]), k


@pytest.mark.parametrize("name", list(CASES))
def test_long_rows_parity(env, name, monkeypatch):
    torch, agp, g, G, sg = env
    a, b, w, eps, kind = CASES[name]
    x = _x(g, kind).astype(np.float32)
    ref, cnt = oracle.propagate(sg, a, b, w, x, eps, 11, wp=32)
    assert cnt["det"].sum() > 4 * 4096
    X = torch.from_numpy(x).to("cuda:0")
    outs = []
    for env_vars in ({}, {"AGP_BIG_ROWS": "0"}, {"AGP_BIG_ROWS": "1"}, {"AGP_AGGREGATION": "binned"},
                     {"AGP_AGGREGATION": "atomic"}):
        for k in ("AGP_BIG_ROWS", "AGP_AGGREGATION"):
            monkeypatch.delenv(k, raising=False)
        for k, v in env_vars.items():
            monkeypatch.setenv(k, v)
        out, st = agp.propagate(G, a, b, w, X, eps, 11, stats=True)
        got = out.cpu().numpy().astype(np.float64)
        _check(got, st, ref, cnt, len(w) - 1)
        outs.append(got)
    assert all(np.array_equal(outs[0], o) for o in outs[1:])


def test_long_rows_binary64(env):
    torch, agp, g, G, sg = env
    a, b, w, eps, kind = CASES["general_signed"]
    x = _x(g, kind).astype(np.float64)
    ref, cnt = oracle.propagate(sg, a, b, w, x, eps, 3, wp=64)
    out, st = agp.propagate(G, a, b, w, torch.from_numpy(x).to("cuda:0"), eps, 3, stats=True)
    _check(out.cpu().numpy(), st, ref, cnt, len(w) - 1)


def test_long_rows_many_columns(env):
    """Every hub in many columns at once: more deferred rows per level than
    a wave has lanes; a column's result does not depend on the others."""
    torch, agp, g, G, sg = env
    a, b, w, eps, _ = CASES["ppr"]
    src = np.array([0, 1, 2, 3] * 10 + list(range(50, 60)))
    x = inputs.one_hot(g.n, src)
    q = np.arange(len(src), dtype=np.uint32) * 3
    ref, cnt = oracle.propagate(sg, a, b, w, x, eps, 5, wp=32, qids=q)
    out, st = agp.propagate(G, a, b, w, torch.from_numpy(x).to("cuda:0"), eps, 5, qids=q, stats=True)
    _check(out.cpu().numpy().astype(np.float64), st, ref, cnt, len(w) - 1)


def test_long_sampled_rows(env, monkeypatch):
    """Hubs reached with a small residue: their sampled suffixes make 8 or
    more work items of 16 windows and, with the deferral cut lowered to 8
    items (AGP_BIG_ITEMS), are deferred to k_samp_big (one item per lane
    over the grid); bit-exact with the oracle in every mode and list
    length, and with the default cut."""
    torch, agp, g, G, sg = env
    monkeypatch.setenv("AGP_BIG_ITEMS", "8")
    deg = np.diff(g.row_ptr)
    rng = np.random.default_rng(3)
    src = []
    for h in (2, 3):  # the hubs of 9000 and 12000 neighbours
        src += [int(v) for v in rng.choice(g.col[g.row_ptr[h]:g.row_ptr[h + 1]], size=3, replace=False)]
    x = inputs.one_hot(g.n, src)
    X = torch.from_numpy(x).to("cuda:0")
    eps = 1e-4
    # TP: level-1 residue of hub h from source s is 1/d_s, so c = 1/(d_s d_h) < eps: sampled, and the row
    # makes ceil(ceil(d_h / 64) / 16) >= 8 items
    for s in src[:1]:
        h = 2
        assert 1.0 / (deg[s] * deg[h]) < eps and ((deg[h] + 63) // 64 + 15) // 16 >= 8
    for a, b, w in ((0.0, 1.0, inputs.weights_tp(6)), (0.5, 0.5, inputs.weights_ppr(0.2, 6))):
        ref, cnt = oracle.propagate(sg, a, b, w, x, eps, 17, wp=32)
        assert cnt["cand"].sum() > 0
        outs = []
        for env_vars in ({}, {"AGP_BIG_ROWS": "0"}, {"AGP_BIG_ROWS": "1"}, {"AGP_AGGREGATION": "binned"},
                         {"AGP_AGGREGATION": "atomic"}, {"AGP_BIG_ITEMS": "64"}):
            for k in ("AGP_BIG_ROWS", "AGP_AGGREGATION"):
                monkeypatch.delenv(k, raising=False)
            monkeypatch.setenv("AGP_BIG_ITEMS", "8")
            for k, v in env_vars.items():
                monkeypatch.setenv(k, v)
            out, st = agp.propagate(G, a, b, w, X, eps, 17, stats=True)
            got = out.cpu().numpy().astype(np.float64)
            _check(got, st, ref, cnt, len(w) - 1)
            outs.append(got)
        assert all(np.array_equal(outs[0], o) for o in outs[1:])
