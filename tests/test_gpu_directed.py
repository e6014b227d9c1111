"""Directed graphs (Section 4, propagation on directed graphs) on the HIP
path, through the C ABI: pushes along out-edges (A~ = A^T) or, reversed,
along in-edges (A~ = A), with out-degree factors.  Graph build, counters and
estimates bit-exact with the oracle."""
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
    g = inputs.directed_chung_lu(6000, 8, 2.2, seed=31)
    return torch, agp, g


MODELS = {
    # (a, b, weights, eps, signal, reverse)
    "ppr": (0.0, 1.0, inputs.weights_ppr(0.2, 15), 1e-5, "onehot", False),
    "hkpr": (0.0, 1.0, inputs.weights_hkpr(4.0, 12), 1e-5, "onehot", False),
    "katz": (0.0, 0.0, inputs.weights_katz(0.02, 10, 0.85), 1e-5, "onehot", False),
    "general_signed": (0.5, 0.5, inputs.weights_ppr(0.1, 8), 1e-4, "normal", False),
    "single_target": (1.0, 0.0, inputs.weights_ppr(0.2, 15), 1e-5, "onehot", True),
    "reverse_general": (0.3, 0.7, inputs.weights_hkpr(2.0, 8), 1e-4, "normal", True),
}


@pytest.mark.parametrize("reverse", [False, True])
def test_directed_graph_build_is_bit_exact(env, reverse):
    torch, agp, g = env
    G = agp.Graph.from_inputs(g, validate=True, directed=True, reverse=reverse)
    rp, col, deg = G.export()
    sg = oracle.directed(g, reverse)
    assert np.array_equal(rp, sg.row_ptr)
    assert np.array_equal(col, sg.col)
    assert np.array_equal(deg, sg.deg)
    assert G.max_degree == int(sg.deg.max())
    if reverse:
        assert not np.array_equal(rp, g.row_ptr)  # really the transpose


@pytest.mark.parametrize("name", list(MODELS))
@pytest.mark.parametrize("C", [1, 9])
def test_directed_parity(env, name, C):
    torch, agp, g = env
    a, b, w, eps, kind, reverse = MODELS[name]
    if kind == "onehot":
        deg_src = np.bincount(g.col, minlength=g.n) if reverse else np.diff(g.row_ptr)
        src = np.random.default_rng(5).choice(np.flatnonzero(deg_src > 0), size=C, replace=False)
        x = inputs.one_hot(g.n, src)
    else:
        x = inputs.features_normal(g.n, C, seed=6)
    G = agp.Graph.from_inputs(g, directed=True, reverse=reverse)
    X = torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")
    out, st = agp.propagate(G, a, b, w, X, eps, 17, stats=True)
    got = out.cpu().numpy().astype(np.float64)
    ref, cnt = oracle.propagate(oracle.directed(g, reverse), a, b, w, x.astype(np.float32), eps, 17, wp=32)
    assert np.array_equal(got, ref), f"max diff {np.abs(got - ref).max()}"
    L = len(w) - 1
    for k in ("frontier", "hash", "det", "cand", "acc", "runs"):
        assert np.array_equal(st[k][: L + 1], cnt[k].sum(axis=0).astype(np.uint64)[: L + 1]), k
    assert st["cand"].sum() > 0


def test_directed_binary64_against_exact_sum(env):
    """binary64 on a directed graph: bit-exact with the oracle, and close to
    the exact truncated sum of the directed Eq. 1."""
    torch, agp, g = env
    a, b, w = 1.0, 0.0, inputs.weights_ppr(0.2, 12)
    t = int(np.argmax(np.bincount(g.col, minlength=g.n)))
    x = inputs.one_hot(g.n, [t]).astype(np.float64)
    G = agp.Graph.from_inputs(g, directed=True, reverse=True)
    out, _ = agp.propagate(G, a, b, w, torch.from_numpy(x).to("cuda:0"), 1e-7, 3)
    got = out.cpu().numpy()[:, 0]
    ref, _ = oracle.propagate(oracle.directed(g, True), a, b, w, x, 1e-7, 3, wp=64)
    assert np.array_equal(got, ref[:, 0])
    exact = _sparse_directed(g, a, b, w, x[:, 0], reverse=True)
    assert np.abs(got - exact).max() <= 1e-3 * np.abs(exact).max()


def _sparse_directed(g, a, b, w, x, reverse):
    import scipy.sparse as sp

    n = g.n
    A = sp.csr_matrix((np.ones(len(g.col)), g.col, g.row_ptr), shape=(n, n))  # A[u, v]: u -> v
    d = np.maximum(np.diff(g.row_ptr), 1).astype(np.float64)
    At = A if reverse else A.T
    P = sp.diags(d ** (-a)) @ At @ sp.diags(d ** (-b))
    acc = w[-1] * x
    for i in range(len(w) - 2, -1, -1):
        acc = w[i] * x + P @ acc
    return acc


def test_directed_flags(env):
    torch, agp, g = env
    rp = np.array([0, 1, 1])
    col = np.array([1])
    with pytest.raises(agp.AGPError) as e:  # asymmetric as an undirected graph
        agp.Graph(rp, col, validate=True)
    assert e.value.code == agp.AGP_EINVAL
    G = agp.Graph(rp, col, validate=True, directed=True)  # fine as a directed one
    assert G.nnz == 1
    with pytest.raises(agp.AGPError):  # reverse needs directed
        agp.Graph(rp, col, reverse=True)
    with pytest.raises(agp.AGPError):  # duplicates still rejected
        agp.Graph(np.array([0, 2, 2]), np.array([1, 1]), validate=True, directed=True)


def test_directed_served_query_equals_batched(env):
    """A single-target query served on the reversed graph equals the batched
    call with the same (seed, query id)."""
    torch, agp, g = env
    G = agp.Graph.from_inputs(g, directed=True, reverse=True)
    w = inputs.weights_ppr(0.2, 10)
    t = int(np.argmax(np.bincount(g.col, minlength=g.n)))
    srv = agp.Server(G, max_slots=2, queue_capacity=4)
    o = torch.zeros(g.n, dtype=torch.float32, device="cuda:0")
    tk = srv.submit(t, 1.0, 0.0, w, 1e-5, 77, 5, o)
    r = None
    import time

    t0 = time.time()
    while r is None and time.time() - t0 < 30:
        r = srv.poll(tk)
    srv.close()
    assert r is not None and r["status"] == agp.AGP_OK
    X = torch.from_numpy(inputs.one_hot(g.n, [t])).to("cuda:0")
    out, _ = agp.propagate(G, 1.0, 0.0, w, X, 1e-5, 77, qids=[5])
    assert torch.equal(out[:, 0], o)
