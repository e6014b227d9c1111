"""Pins of the oracle's local clustering sweep (Section 5: nodes sorted by
pi(v)/d_v descending, the prefix of minimum conductance
Phi(S) = |cut(S)| / min(vol(S), 2m - vol(S)))."""
import math

import numpy as np
import pytest

from paper_2106_03058_amd import inputs


def _definition(g, pi):
    """The sweep written out from the definitions: a sort by an explicit key,
    then cut and volume of every prefix recounted over all arcs."""
    n = g.n
    deg = np.diff(g.row_ptr)
    rows = np.repeat(np.arange(n), deg)

    def key(v):
        iso = deg[v] == 0
        r = pi[v] / deg[v] if deg[v] > 0 else 0.0
        return (iso, -r, v)

    order = sorted(range(n), key=key)
    two_m = int(g.row_ptr[-1])
    best, best_phi = 0, math.inf
    in_s = np.zeros(n, dtype=bool)
    for i in range(n - 1):
        in_s[order[i]] = True
        cut = int(np.sum(in_s[rows] & ~in_s[g.col]))  # arcs leaving S (loops never do)
        vol = int(deg[in_s].sum())
        denom = min(vol, two_m - vol)
        if denom > 0 and cut / denom < best_phi:
            best_phi, best = cut / denom, i + 1
    return best, best_phi, np.array(order)


@pytest.mark.parametrize("seed", [1, 2, 3])
@pytest.mark.parametrize("loops", [False, True])
def test_sweep_matches_the_definition(orc, seed, loops):
    g = inputs.chung_lu(150, 4, 2.5, seed=seed, self_loops=loops)
    rng = np.random.default_rng(seed)
    pi = rng.random(g.n) * (rng.random(g.n) < 0.4)  # a sparse estimate, many zeros
    pi[:5] = pi[5]  # ties
    size, phi, order = orc.sweep(g, pi)
    ref_size, ref_phi, ref_order = _definition(g, pi)
    assert np.array_equal(order, ref_order)
    assert size == ref_size and phi == ref_phi


def test_sweep_finds_the_clique_behind_a_bridge(orc):
    """Two k-cliques joined by one edge, the estimate on the first clique: the
    minimum-conductance prefix is that clique, Phi = 1 / (k (k - 1) + 1)."""
    k = 12
    src, dst = [], []
    for base in (0, k):
        for i in range(k):
            for j in range(i + 1, k):
                src.append(base + i)
                dst.append(base + j)
    src.append(0)
    dst.append(k)
    g = inputs.csr_from_pairs(2 * k, np.array(src), np.array(dst))
    pi = np.zeros(2 * k)
    pi[:k] = np.linspace(1.0, 0.5, k)
    size, phi, order = orc.sweep(g, pi)
    assert size == k
    assert set(order[:k].tolist()) == set(range(k))
    assert phi == 1.0 / (k * (k - 1) + 1)


def test_sweep_isolated_nodes_and_degenerate_sizes(orc):
    g = inputs.Graph(5, np.array([0, 1, 2, 2, 2, 2]), np.array([1, 0], dtype=np.int32))  # edge 0-1, 3 isolated
    size, phi, order = orc.sweep(g, np.array([0.0, 0.0, 9.0, 9.0, 9.0]))
    assert list(order[:2]) == [0, 1]  # isolated nodes last even with larger pi
    assert size == 1 and phi == 1.0  # S = {0}: one cut arc, vol 1
    g1 = inputs.Graph(1, np.array([0, 0]), np.array([], dtype=np.int32))
    size, phi, _ = orc.sweep(g1, np.array([1.0]))
    assert size == 0 and math.isinf(phi)
