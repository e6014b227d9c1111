"""Parity of the HIP path with the CPU oracle, through the C ABI.

Integer results (sorted CSR, degrees, per-level frontier sizes and hashes,
deterministic / candidate / accepted push counts) must be bit-exact.  The
floating point estimates must agree within 1e-5 relative or 1e-9 absolute
per entry; by construction (same decisions, exact level sums, the same
rounding) they are in fact bit-identical, which is also asserted.
"""
import numpy as np
import pytest

import oracle
from oracle import dense
from paper_2106_03058_amd import inputs

pytestmark = pytest.mark.gpu

RTOL, ATOL = 1e-5, 1e-9


@pytest.fixture(scope="module")
def torch_dev():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch, torch.device("cuda:0")


@pytest.fixture(scope="module")
def agp(torch_dev):
    from paper_2106_03058_amd import agp as _agp

    _agp.lib()
    return _agp


def _run(agp, torch_dev, g, a, b, w, x, eps, seed, *, wp=32, qids=None, self_loops=False, G=None):
    torch, dev = torch_dev
    if G is None:
        G = agp.Graph.from_inputs(g, validate=True, self_loops=self_loops)
    dt = torch.float32 if wp == 32 else torch.float64
    X = torch.from_numpy(np.ascontiguousarray(x)).to(dev, dt)
    out, st = agp.propagate(G, a, b, w, X, eps, seed, qids=qids, stats=True)
    return out.cpu().numpy().astype(np.float64), st


def _oracle(g, a, b, w, x, eps, seed, *, wp=32, qids=None):
    sg = oracle.degree_sort(g)
    xx = np.asarray(x, dtype=np.float32 if wp == 32 else np.float64)
    return oracle.propagate(sg, a, b, w, xx, eps, seed, wp=wp, qids=qids)


def _assert_parity(got, st, ref, cnt, L):
    assert got.shape == ref.shape
    bad = ~np.isclose(got, ref, rtol=RTOL, atol=ATOL)
    assert not bad.any(), f"{bad.sum()} entries outside tolerance, max diff {np.abs(got - ref).max()}"
    assert np.array_equal(got, ref), f"not bit-identical: max diff {np.abs(got - ref).max()}"
    for k in ("frontier", "hash", "det", "cand", "acc", "runs"):
        want = cnt[k].sum(axis=0).astype(np.uint64)  # summed over columns (hash mod 2^64)
        assert np.array_equal(st[k][: L + 1], want[: L + 1]), f"counter {k}: {st[k]} vs {want}"


# ------------------------------------------------------------ graph build

@pytest.mark.parametrize("loops", [False, True])
def test_degree_sorted_csr_is_bit_exact(agp, torch_dev, loops):
    g = inputs.chung_lu(20000, 12, 2.2, seed=3)  # hub rows longer than one LDS tile
    G = agp.Graph.from_inputs(g, validate=True, self_loops=loops)
    rp, col, deg = G.export()
    gl = inputs.csr_from_pairs(g.n, *_pairs(g), self_loops=True) if loops else g
    sg = oracle.degree_sort(gl)
    assert np.array_equal(rp, sg.row_ptr)
    assert np.array_equal(col, sg.col)
    assert np.array_equal(deg, sg.deg)
    assert G.max_degree == int(sg.deg.max())
    assert G.max_degree > 64
    # degree groups floor(log2 d_v) of every arc, from the oracle's sorted rows
    gid = G.groups()
    want = np.floor(np.log2(sg.fdeg[sg.col].astype(np.float64))).astype(np.uint8)
    assert np.array_equal(gid, want)
    for u in range(0, g.n, 997):  # non-decreasing along rows
        assert np.all(np.diff(gid[rp[u]:rp[u + 1]].astype(np.int32)) >= 0)


def _pairs(g):
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    return rows, g.col.astype(np.int64)


def test_star_hub_row(agp, torch_dev):
    g = inputs.star_graph(50000)
    G = agp.Graph.from_inputs(g, validate=True)
    rp, col, deg = G.export()
    sg = oracle.degree_sort(g)
    assert np.array_equal(col, sg.col) and np.array_equal(deg, sg.deg)


def test_invalid_graphs_rejected(agp, torch_dev):
    # asymmetric
    with pytest.raises(agp.AGPError) as e:
        agp.Graph(np.array([0, 1, 1]), np.array([1]), validate=True)
    assert e.value.code == agp.AGP_EINVAL
    # duplicate arc
    with pytest.raises(agp.AGPError):
        agp.Graph(np.array([0, 2, 4]), np.array([1, 1, 0, 0]), validate=True)
    # id out of range
    with pytest.raises(agp.AGPError):
        agp.Graph(np.array([0, 1, 2]), np.array([1, 5]))
    # empty graph is fine
    G = agp.Graph(np.array([0]), np.array([], dtype=np.int32))
    assert G.n == 0 and G.nnz == 0


# ------------------------------------------------------------ propagation

CASES = {
    # name: (a, b, weights, eps, signal)
    "ppr": (0.0, 1.0, inputs.weights_ppr(0.2, 20), 1e-5, "onehot"),
    "katz": (0.0, 0.0, None, 1e-6, "onehot"),
    "tp": (0.0, 1.0, inputs.weights_tp(10), 1e-5, "onehot"),
    "hkpr": (0.0, 1.0, inputs.weights_hkpr(5.0, 15), 1e-5, "onehot"),
    "gdc_signed": (0.5, 0.5, inputs.weights_hkpr(5.0, 10), 1e-4, "normal"),
    "appnp_uniform": (0.5, 0.5, inputs.weights_ppr(0.1, 10), 1e-4, "uniform"),
    "single_target": (1.0, 0.0, inputs.weights_ppr(0.2, 10), 1e-5, "onehot"),
    "general_ab": (0.3, 0.7, inputs.weights_hkpr(2.0, 8), 1e-4, "normal"),
}


def _signal(g, kind, C, seed):
    if kind == "onehot":
        return inputs.one_hot(g.n, inputs.sources_uniform(g, C, seed))
    if kind == "normal":
        return inputs.features_normal(g.n, C, seed)
    return inputs.features_uniform(g.n, C, -1.0, 1.0, seed)


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("C", [1, 5, 70])
def test_propagate_parity_fp32(agp, torch_dev, name, C):
    a, b, w, eps, kind = CASES[name]
    g = inputs.chung_lu(3000, 10, 2.5, seed=17, self_loops=kind != "onehot")
    if w is None:
        lam = inputs.lambda_max(g)
        w = inputs.weights_katz(0.85 / lam, 30, 0.85)
    x = _signal(g, kind, C, seed=C)
    got, st = _run(agp, torch_dev, g, a, b, w, x, eps, seed=99)
    ref, cnt = _oracle(g, a, b, w, x, eps, 99)
    _assert_parity(got, st, ref, cnt, len(w) - 1)
    assert st["pushes"] > 0


@pytest.mark.parametrize("zero_share", [0.1, 0.49, 0.51, 0.9])
@pytest.mark.parametrize("wp", [32, 64])
def test_signals_with_zero_cells(agp, torch_dev, zero_share, wp):
    """Level 0 visits every cell of a mostly non-zero signal and skips its
    zeros, and lists the non-zero cells of a mostly zero one: either way the
    frontier, the counters and the estimates are the oracle's."""
    g = inputs.chung_lu(3000, 10, 2.5, seed=23, self_loops=True)
    x = inputs.features_uniform(g.n, 6, -1.0, 1.0, seed=24)
    rng = np.random.default_rng(25)
    x[rng.random(x.shape) < zero_share] = 0.0
    x[5, :] = 0.0  # a node with no signal at all
    x = x.astype(np.float32 if wp == 32 else np.float64)
    w = inputs.weights_ppr(0.1, 8)
    got, st = _run(agp, torch_dev, g, 0.5, 0.5, w, x, 1e-4, 31, wp=wp)
    ref, cnt = _oracle(g, 0.5, 0.5, w, x, 1e-4, 31, wp=wp)
    _assert_parity(got, st, ref, cnt, 8)
    assert st["frontier"][0] == np.count_nonzero(x)


@pytest.mark.parametrize("kind", ["normal", "sparse", "onehot", "tiny"])
@pytest.mark.parametrize("wp", [32, 64])
def test_one_column_signals(agp, torch_dev, kind, wp):
    """One column over several 4096-row threshold blocks with a ragged tail:
    the one-column threshold pass gives the sum in row order (exact sums of
    binary32 blocks taken in any order; one entry of 1e-30, or binary64
    entries, make the block sums inexact and the wave adds in row order), so
    theta, the level-0 frontier and the estimates are the oracle's; a
    non-finite entry in the last block is rejected."""
    torch, dev = torch_dev
    g = inputs.chung_lu(10000, 8, 2.5, seed=41, self_loops=kind != "onehot")
    if kind == "onehot":
        x = inputs.one_hot(g.n, [9999])
    else:
        x = inputs.features_normal(g.n, 1, seed=42)
        if kind == "sparse":
            x[np.random.default_rng(43).random(x.shape) < 0.9] = 0.0
        if kind == "tiny":
            x[7000, 0] = 1e-30
    x = x.astype(np.float32 if wp == 32 else np.float64)
    w = inputs.weights_ppr(0.2, 8)
    got, st = _run(agp, torch_dev, g, 0.5, 0.5, w, x, 1e-5, 44, wp=wp)
    ref, cnt = _oracle(g, 0.5, 0.5, w, x, 1e-5, 44, wp=wp)
    _assert_parity(got, st, ref, cnt, 8)
    assert st["frontier"][0] == np.count_nonzero(x)
    xn = torch.from_numpy(x.copy()).to(dev)
    xn[9000, 0] = float("inf")
    with pytest.raises(agp.AGPError) as e:
        agp.propagate(agp.Graph.from_inputs(g), 0.5, 0.5, w, xn, 1e-5, 44)
    assert e.value.code == agp.AGP_EINVAL


def test_parity_fp64_c1_shape(agp, torch_dev):
    """PPR from node 0 (the top-weight hub) on a Chung-Lu graph, binary64."""
    g = inputs.chung_lu(10000, 10, 2.5, seed=1)
    w = inputs.weights_ppr(0.2, 20)
    x = inputs.one_hot(g.n, [0]).astype(np.float64)
    got, st = _run(agp, torch_dev, g, 0.0, 1.0, w, x, 1e-6, seed=1, wp=64)
    ref, cnt = _oracle(g, 0.0, 1.0, w, x, 1e-6, 1, wp=64)
    _assert_parity(got, st, ref, cnt, 20)
    # error against the exact truncated sum (eps = 0 oracle, binary64)
    exact, _ = _oracle(g, 0.0, 1.0, w, x, 0.0, 1, wp=64)
    err = np.abs(got[:, 0] - exact[:, 0])
    L = 20
    # Lemma 3.2: sd <= sqrt(L(L+1) eps / 2 * pi(v)); check the well-resolved entries
    big = exact[:, 0] >= 1e-3
    sd = np.sqrt(L * (L + 1) * 1e-6 / 2 * exact[big, 0])
    assert big.sum() > 10 and np.all(err[big] <= 6 * sd)


def test_fp64_signed(agp, torch_dev):
    g = inputs.chung_lu(2000, 8, 2.5, seed=5, self_loops=True)
    w = inputs.weights_hkpr(4.0, 8)
    x = inputs.features_normal(g.n, 3, seed=2).astype(np.float64)
    got, st = _run(agp, torch_dev, g, 0.5, 0.5, w, x, 1e-4, seed=4, wp=64)
    ref, cnt = _oracle(g, 0.5, 0.5, w, x, 1e-4, 4, wp=64)
    _assert_parity(got, st, ref, cnt, 8)


def test_hubs_and_many_windows(agp, torch_dev):
    # star with 20000 leaves: the hub row spans 313 sampling windows
    g = inputs.star_graph(20000)
    x = inputs.one_hot(g.n, [0, 1, 2])
    for eps, w in ((1e-3, inputs.weights_tp(4)), (1e-6, inputs.weights_ppr(0.3, 6))):
        got, st = _run(agp, torch_dev, g, 0.0, 1.0, w, x, eps, seed=5)
        ref, cnt = _oracle(g, 0.0, 1.0, w, x, eps, 5)
        _assert_parity(got, st, ref, cnt, len(w) - 1)
    got, st = _run(agp, torch_dev, g, 0.5, 0.5, inputs.weights_ppr(0.2, 5), x, 1e-3, seed=6)
    ref, cnt = _oracle(g, 0.5, 0.5, inputs.weights_ppr(0.2, 5), x, 1e-3, 6)
    _assert_parity(got, st, ref, cnt, 5)


@pytest.mark.parametrize("a, b", [(0.0, 1.0), (0.5, 0.5)])
def test_batches_with_many_work_items(agp, torch_dev, a, b):
    """Sixteen leaf sources of a 20000-leaf star: at level 1 the hub holds
    a residue in all 16 columns, each a work item per 16 sampling windows
    (20 items), so a batch holds more work items than the level kernel maps
    to their entries in LDS and the rest are found by search."""
    g = inputs.star_graph(20000)
    x = inputs.one_hot(g.n, list(range(1, 17)))
    w = inputs.weights_ppr(0.2, 4)
    got, st = _run(agp, torch_dev, g, a, b, w, x, 1e-3, seed=8)
    ref, cnt = _oracle(g, a, b, w, x, 1e-3, 8)
    _assert_parity(got, st, ref, cnt, 4)
    assert st["cand"][1] > 16 * 100  # the hub's columns were sampled, not pushed deterministically


def test_edge_cases(agp, torch_dev):
    g = inputs.chung_lu(1500, 6, 2.5, seed=8)
    deg = g.degree
    iso = np.flatnonzero(deg == 0)
    w = inputs.weights_ppr(0.2, 6)
    x = inputs.one_hot(g.n, [int(np.argmax(deg)), 3, 4])
    x[:, 1] = 0.0  # an empty column
    if iso.size:
        x[:, 2] = 0.0
        x[iso[0], 2] = 1.0  # mass on an isolated node stays in its reserve
    for L, eps in ((0, 1e-3), (1, 1e-3), (6, 1e-9), (6, 0.5)):
        ww = w[: L + 1]
        got, st = _run(agp, torch_dev, g, 0.0, 1.0, ww, x, eps, seed=11)
        ref, cnt = _oracle(g, 0.0, 1.0, ww, x, eps, 11)
        _assert_parity(got, st, ref, cnt, L)


def test_determinism_and_qids(agp, torch_dev):
    g = inputs.chung_lu(4000, 10, 2.5, seed=9)
    w = inputs.weights_ppr(0.2, 15)
    src = inputs.sources_uniform(g, 8, seed=3)
    x = inputs.one_hot(g.n, src)
    G = agp.Graph.from_inputs(g)
    a1, s1 = _run(agp, torch_dev, g, 0.0, 1.0, w, x, 1e-5, seed=21, G=G)
    a2, s2 = _run(agp, torch_dev, g, 0.0, 1.0, w, x, 1e-5, seed=21, G=G)
    assert np.array_equal(a1, a2)
    # column 5 alone, with its batch qid, equals its value inside the batch
    alone, _ = _run(agp, torch_dev, g, 0.0, 1.0, w, x[:, 5:6], 1e-5, seed=21, qids=[5], G=G)
    assert np.array_equal(alone[:, 0], a1[:, 5])
    other, _ = _run(agp, torch_dev, g, 0.0, 1.0, w, x, 1e-5, seed=22, G=G)
    assert not np.array_equal(other, a1)


def test_error_paths(agp, torch_dev):
    torch, dev = torch_dev
    g = inputs.chung_lu(500, 6, 2.5, seed=2)
    G = agp.Graph.from_inputs(g)
    x = torch.from_numpy(inputs.one_hot(g.n, [0])).to(dev)
    w = inputs.weights_ppr(0.2, 5)
    with pytest.raises(agp.AGPError) as e:
        agp.propagate(G, 0.0, 1.0, w, x, 0.0, 1)
    assert e.value.code == agp.AGP_ENOTSUP
    for kw in (dict(a=2.0), dict(eps=-1.0), dict(w=np.ones(300)), dict(w=-w)):
        args = dict(a=0.0, eps=1e-3, w=w) | kw
        with pytest.raises(agp.AGPError) as e:
            agp.propagate(G, args["a"], 1.0, args["w"], x, args["eps"], 1)
        assert e.value.code == agp.AGP_EINVAL
    xn = x.clone()
    xn[3, 0] = float("nan")
    with pytest.raises(agp.AGPError) as e:
        agp.propagate(G, 0.0, 1.0, w, xn, 1e-3, 1)
    assert e.value.code == agp.AGP_EINVAL
    # a threshold so small that a push exceeds the exact accumulator range
    with pytest.raises(agp.AGPError) as e:
        agp.propagate(G, 0.0, 1.0, w, x, 1e-16, 1)
    assert e.value.code == agp.AGP_ERANGE
    # the library recovers: a normal call afterwards still matches the oracle
    got, st = _run(agp, torch_dev, g, 0.0, 1.0, w, inputs.one_hot(g.n, [0]), 1e-4, seed=3, G=G)
    ref, cnt = _oracle(g, 0.0, 1.0, w, inputs.one_hot(g.n, [0]), 1e-4, 3)
    _assert_parity(got, st, ref, cnt, 5)


@pytest.mark.parametrize("name", ["gdc_signed", "general_ab", "single_target"])
def test_factor_vectors_are_bit_identical(agp, torch_dev, name, monkeypatch):
    """The per-call node and arc factor vectors give the results and counters
    of reading the factors through the degree tables (and the oracle's)."""
    a, b, w, eps, kind = CASES[name]
    g = inputs.chung_lu(3000, 10, 2.5, seed=29, self_loops=kind != "onehot")
    x = _signal(g, kind, 24, seed=30)
    ref, cnt = _oracle(g, a, b, w, x, eps, 31)
    monkeypatch.setenv("AGP_FACTOR_VECTORS", "0")
    got0, st0 = _run(agp, torch_dev, g, a, b, w, x, eps, seed=31)
    monkeypatch.delenv("AGP_FACTOR_VECTORS")
    got1, st1 = _run(agp, torch_dev, g, a, b, w, x, eps, seed=31)
    _assert_parity(got0, st0, ref, cnt, len(w) - 1)
    _assert_parity(got1, st1, ref, cnt, len(w) - 1)


@pytest.mark.parametrize("name", ["ppr", "tp", "gdc_signed", "general_ab"])
def test_aggregation_modes_are_bit_identical(agp, torch_dev, name, monkeypatch):
    """Binned LDS aggregation, its record-overflow fallback and plain atomics
    give the same bits (exact integer sums), equal to the oracle's; so do
    records kept in two column groups (cells local to a group, as when n C
    reaches 2^31; 33 columns: groups of 17 and 16), with and without
    overflow."""
    a, b, w, eps, kind = CASES[name]
    g = inputs.chung_lu(6000, 12, 2.5, seed=31, self_loops=kind != "onehot")
    x = _signal(g, kind, 33, seed=4)
    G = agp.Graph.from_inputs(g)
    ref, cnt = _oracle(g, a, b, w, x, eps, 5)
    results = []
    for env in ({}, {"AGP_AGGREGATION": "atomic"}, {"AGP_AGGREGATION": "binned"}, {"AGP_AGGREGATION": "auto"},
                {"AGP_AGGREGATION": "binned", "AGP_RECORD_CAP": "5000"},
                {"AGP_AGGREGATION": "binned", "AGP_RECORD_GROUPS": "2"},
                {"AGP_AGGREGATION": "auto", "AGP_RECORD_GROUPS": "2"},
                {"AGP_AGGREGATION": "binned", "AGP_RECORD_GROUPS": "2", "AGP_RECORD_CAP": "5000"}):
        for k in ("AGP_AGGREGATION", "AGP_RECORD_CAP", "AGP_RECORD_GROUPS"):
            monkeypatch.delenv(k, raising=False)
        for k, v in env.items():
            monkeypatch.setenv(k, v)
        got, st = _run(agp, torch_dev, g, a, b, w, x, eps, seed=5, G=G)
        _assert_parity(got, st, ref, cnt, len(w) - 1)
        results.append(got)
    assert all(np.array_equal(results[0], r) for r in results[1:])


def test_autotune_keeps_results(agp, torch_dev):
    """Every autotuned choice gives the same bits; the pick is reused."""
    torch, dev = torch_dev
    g = inputs.chung_lu(5000, 10, 2.5, seed=41)
    G = agp.Graph.from_inputs(g)
    x = inputs.one_hot(g.n, inputs.sources_uniform(g, 40, seed=6))
    w = inputs.weights_ppr(0.2, 12)
    X = torch.from_numpy(x).to(dev)
    before = agp.get_tuning(G, 40, 0.0, 1.0)
    assert before == {"aggregation": "auto", "level_blocks": 4096, "dense": "never", "tile_columns": 0,
                      "big_row": 4096, "big_items": 64, "sparse_shift": 5, "bin_shift": 3, "capture": 0}
    out = torch.empty_like(X)
    pick = agp.autotune(G, 0.0, 1.0, w, X, 1e-5, 9, out=out)
    assert agp.get_tuning(G, 40, 0.0, 1.0) == pick
    ref, _ = _oracle(g, 0.0, 1.0, w, x, 1e-5, 9)
    assert np.array_equal(out.cpu().numpy().astype(np.float64), ref)
    again, _ = agp.propagate(G, 0.0, 1.0, w, X, 1e-5, 9)
    assert np.array_equal(again.cpu().numpy().astype(np.float64), ref)


@pytest.mark.parametrize("name,wp,tile", [("appnp_uniform", 32, "7"), ("ppr", 32, "5"), ("gdc_signed", 64, "3")])
def test_column_tiles_are_bit_identical(agp, torch_dev, name, wp, tile, monkeypatch):
    """A call split into column tiles (the last one ragged) gives the bits of
    the untiled call and of the oracle: column c keeps its own random streams."""
    a, b, w, eps, kind = CASES[name]
    g = inputs.chung_lu(4000, 12, 2.5, seed=37, self_loops=kind != "onehot")
    x = _signal(g, kind, 33, seed=8)
    G = agp.Graph.from_inputs(g)
    ref, cnt = _oracle(g, a, b, w, x, eps, 6, wp=wp)
    monkeypatch.delenv("AGP_COLUMN_TILE", raising=False)
    whole, st_whole = _run(agp, torch_dev, g, a, b, w, x, eps, seed=6, wp=wp, G=G)
    monkeypatch.setenv("AGP_COLUMN_TILE", tile)
    tiled, st_tiled = _run(agp, torch_dev, g, a, b, w, x, eps, seed=6, wp=wp, G=G)
    _assert_parity(tiled, st_tiled, ref, cnt, len(w) - 1)
    assert np.array_equal(whole, tiled)
    # explicit qids follow their columns into the tiles
    q = np.arange(500, 533, dtype=np.uint32)[::-1].copy()
    ref_q, _ = _oracle(g, a, b, w, x, eps, 6, wp=wp, qids=q)
    tiled_q, _ = _run(agp, torch_dev, g, a, b, w, x, eps, seed=6, wp=wp, G=G, qids=q)
    assert np.array_equal(tiled_q, ref_q)
