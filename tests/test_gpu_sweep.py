"""Local clustering sweep (Section 5, the quality of local clusters) on the
HIP path, through the C ABI: the node order, the best prefix size and its
conductance bit-exact with the oracle's sweep of the same estimate."""
import math

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
    return torch, agp


def _sweep_both(torch, agp, g, pi, *, self_loops=False):
    G = agp.Graph.from_inputs(g, self_loops=self_loops)
    p32 = np.ascontiguousarray(pi, dtype=np.float32)
    size, phi, order = agp.sweep(G, torch.from_numpy(p32).to("cuda:0"))
    og = inputs.add_self_loops(g.n, g.row_ptr, g.col) if self_loops else g
    ref = oracle.sweep(og, p32.astype(np.float64))
    return (size, phi, order.cpu().numpy()), ref


def _assert_same(got, ref):
    size, phi, order = got
    rsize, rphi, rorder = ref
    assert np.array_equal(order, rorder), f"first difference at {np.flatnonzero(order != rorder)[:5]}"
    assert size == rsize
    assert phi == rphi or (math.isinf(phi) and math.isinf(rphi))


def _sparse_pi(n, seed, density=0.3):
    rng = np.random.default_rng(seed)
    pi = (rng.random(n) * (rng.random(n) < density)).astype(np.float32)
    pi[: min(n, 20)] = pi[min(n - 1, 20)]  # ties
    return pi


@pytest.mark.parametrize("n,seed,loops", [(300, 1, False), (300, 2, True), (5000, 3, False), (70000, 4, True)])
def test_sweep_parity_random_estimate(env, n, seed, loops):
    torch, agp = env
    g = inputs.chung_lu(n, 6, 2.3, seed=seed)
    got, ref = _sweep_both(torch, agp, g, _sparse_pi(n, seed), self_loops=loops)
    _assert_same(got, ref)
    assert 1 <= got[0] <= n - 1


def test_sweep_parity_on_a_heat_kernel_estimate(env):
    """The use of Section 5: sweep a heat kernel PageRank estimate from one
    seed node (the estimate computed by the oracle)."""
    torch, agp = env
    g = inputs.chung_lu(20000, 10, 2.1, seed=8)
    deg = np.diff(g.row_ptr)
    s = int(np.flatnonzero(deg > 0)[7])
    w = inputs.weights_hkpr(5.0, 20)
    pi, _ = oracle.propagate(oracle.degree_sort(g), 0.0, 1.0, w, inputs.one_hot(g.n, [s]), 1e-6, 11, wp=32)
    got, ref = _sweep_both(torch, agp, g, pi[:, 0])
    _assert_same(got, ref)
    assert got[0] >= 1


def test_sweep_full_size(env):
    """A power-law graph of 2^21 nodes and about 2 * 10^7 arcs with a sparse
    estimate on it: every position of the order, the size and Phi."""
    torch, agp = env
    g = inputs.chung_lu(1 << 21, 10, 2.1, seed=12)
    pi = _sparse_pi(g.n, 12, density=0.05)
    got, ref = _sweep_both(torch, agp, g, pi)
    _assert_same(got, ref)


def test_sweep_signed_and_zero_values(env):
    """Negative and zero estimates sort after the positive ones (descending
    pi/d), -0 and +0 as one value."""
    torch, agp = env
    g = inputs.chung_lu(2000, 5, 2.5, seed=21)
    rng = np.random.default_rng(21)
    pi = rng.normal(size=g.n).astype(np.float32)
    pi[rng.random(g.n) < 0.2] = 0.0
    pi[rng.random(g.n) < 0.1] = -0.0
    got, ref = _sweep_both(torch, agp, g, pi)
    _assert_same(got, ref)


def test_sweep_bridged_cliques(env):
    torch, agp = env
    k = 16
    src, dst = [], []
    for base in (0, k):
        for i in range(k):
            for j in range(i + 1, k):
                src.append(base + i)
                dst.append(base + j)
    src.append(0)
    dst.append(k)
    g = inputs.csr_from_pairs(2 * k, np.array(src), np.array(dst))
    pi = np.zeros(2 * k, dtype=np.float32)
    pi[:k] = np.linspace(1.0, 0.5, k)
    (size, phi, order), ref = _sweep_both(torch, agp, g, pi)
    _assert_same((size, phi, order), ref)
    assert size == k and phi == 1.0 / (k * (k - 1) + 1)


def test_sweep_degenerate_graphs(env):
    torch, agp = env
    # edge 0-1 and three isolated nodes with the largest estimates
    g = inputs.Graph(5, np.array([0, 1, 2, 2, 2, 2]), np.array([1, 0], dtype=np.int32))
    got, ref = _sweep_both(torch, agp, g, np.array([0.0, 0.0, 9.0, 9.0, 9.0]))
    _assert_same(got, ref)
    assert list(got[2][:2]) == [0, 1] and got[0] == 1 and got[1] == 1.0
    # no arcs at all: no prefix has a conductance
    g0 = inputs.Graph(4, np.zeros(5, dtype=np.int64), np.array([], dtype=np.int32))
    got, ref = _sweep_both(torch, agp, g0, np.ones(4))
    _assert_same(got, ref)
    assert got[0] == 0 and math.isinf(got[1])
    # one node
    g1 = inputs.Graph(1, np.array([0, 0]), np.array([], dtype=np.int32))
    G1 = agp.Graph.from_inputs(g1)
    size, phi, order = agp.sweep(G1, torch.ones(1, device="cuda:0"))
    assert size == 0 and math.isinf(phi) and order.numel() == 1


def test_sweep_without_order_and_errors(env):
    torch, agp = env
    g = inputs.chung_lu(1000, 4, 2.5, seed=5)
    G = agp.Graph.from_inputs(g)
    pi = torch.from_numpy(_sparse_pi(g.n, 5)).to("cuda:0")
    size, phi, order = agp.sweep(G, pi, order=False)
    s2, p2, _ = agp.sweep(G, pi)
    assert order is None and (size, phi) == (s2, p2)
    with pytest.raises(ValueError):
        agp.sweep(G, pi[:-1])
    d = inputs.directed_chung_lu(500, 4, 2.5, seed=6)
    D = agp.Graph.from_inputs(d, directed=True)
    with pytest.raises(agp.AGPError) as e:
        agp.sweep(D, torch.zeros(d.n, device="cuda:0"))
    assert e.value.code == agp.AGP_EINVAL


def test_sweep_of_strided_columns(env):
    """Columns of a row-major n x C result are swept in place (stride C) and
    give what the contiguous copies give."""
    torch, agp = env
    g = inputs.chung_lu(4000, 6, 2.3, seed=41)
    G = agp.Graph.from_inputs(g)
    P = torch.from_numpy(np.stack([_sparse_pi(g.n, 41 + c) for c in range(5)], axis=1)).to("cuda:0")
    for c in range(5):
        s1, p1, o1 = agp.sweep(G, P[:, c])
        s2, p2, o2 = agp.sweep(G, P[:, c].contiguous())
        assert (s1, p1) == (s2, p2) and torch.equal(o1, o2)
        _assert_same((s1, p1, o1.cpu().numpy()), oracle.sweep(g, P[:, c].cpu().numpy().astype(np.float64)))


@pytest.mark.parametrize("n,C,loops", [(300, 5, False), (4000, 64, True), (20000, 70, False)])
def test_sweep_batch_equals_the_oracle(env, n, C, loops):
    """The batched sweep (groups of up to 64 columns, one segmented sort and
    one arc pass per group) gives every column's size and Phi bit-exact."""
    torch, agp = env
    g = inputs.chung_lu(n, 6, 2.3, seed=C)
    G = agp.Graph.from_inputs(g, self_loops=loops)
    og = inputs.add_self_loops(g.n, g.row_ptr, g.col) if loops else g
    P = np.stack([_sparse_pi(n, 100 + c, density=0.05 + 0.9 * (c % 3) / 2) for c in range(C)], axis=1)
    P[:, 1] = 0.0  # a column without estimate: all ties, order by id
    size, phi = agp.sweep_batch(G, torch.from_numpy(P).to("cuda:0"))
    for c in range(C):
        rs, rphi, _ = oracle.sweep(og, P[:, c].astype(np.float64))
        assert (size[c], phi[c]) == (rs, rphi) or (size[c] == rs == 0 and math.isinf(phi[c])), c


def test_sweep_batch_of_propagation_columns(env):
    """Heat-kernel estimates of 40 seeds (computed by the oracle) swept in
    one call, as strided columns of the n x 48 block they sit in."""
    torch, agp = env
    g = inputs.chung_lu(30000, 10, 2.1, seed=9)
    s = np.random.default_rng(3).choice(np.flatnonzero(np.diff(g.row_ptr) > 0), size=48, replace=False)
    ref, _ = oracle.propagate(oracle.degree_sort(g), 0.0, 1.0, inputs.weights_hkpr(5.0, 15),
                              inputs.one_hot(g.n, s), 1e-5, 4, wp=32)
    G = agp.Graph.from_inputs(g)
    X = torch.from_numpy(ref.astype(np.float32)).to("cuda:0")
    size, phi = agp.sweep_batch(G, X[:, 8:48])
    for c in range(40):
        rs, rphi, _ = oracle.sweep(g, ref[:, 8 + c])
        assert (size[c], phi[c]) == (rs, rphi), c


def test_sweep_batch_full_size(env):
    """64 sparse estimates on a 2^20-node power-law graph: size and Phi of
    every column against the oracle (a sample of 8) and against agp_sweep."""
    torch, agp = env
    g = inputs.chung_lu(1 << 20, 12, 2.1, seed=17)
    G = agp.Graph.from_inputs(g)
    P = torch.from_numpy(np.stack([_sparse_pi(g.n, 500 + c, density=0.1) for c in range(64)], axis=1)).to("cuda:0")
    size, phi = agp.sweep_batch(G, P)
    for c in range(64):
        s1, p1, _ = agp.sweep(G, P[:, c], order=False)
        assert (size[c], phi[c]) == (s1, p1), c
    for c in range(0, 64, 8):
        rs, rphi, _ = oracle.sweep(g, P[:, c].cpu().numpy().astype(np.float64))
        assert (size[c], phi[c]) == (rs, rphi), c


def test_sweep_batch_degenerate(env):
    torch, agp = env
    g1 = inputs.Graph(1, np.array([0, 0]), np.array([], dtype=np.int32))
    size, phi = agp.sweep_batch(agp.Graph.from_inputs(g1), torch.ones((1, 3), device="cuda:0"))
    assert list(size) == [0, 0, 0] and np.all(np.isinf(phi))
    g0 = inputs.Graph(4, np.zeros(5, dtype=np.int64), np.array([], dtype=np.int32))
    size, phi = agp.sweep_batch(agp.Graph.from_inputs(g0), torch.ones((4, 2), device="cuda:0"))
    assert list(size) == [0, 0] and np.all(np.isinf(phi))
    g = inputs.chung_lu(500, 4, 2.5, seed=2)
    G = agp.Graph.from_inputs(g)
    with pytest.raises(ValueError):
        agp.sweep_batch(G, torch.ones((500, 4), device="cuda:0").t())  # columns not contiguous in rows
    d = inputs.directed_chung_lu(300, 4, 2.5, seed=6)
    with pytest.raises(agp.AGPError):
        agp.sweep_batch(agp.Graph.from_inputs(d, directed=True), torch.zeros((300, 2), device="cuda:0"))
