"""Dense FP64 closed forms of graph propagation -- TEST INFRASTRUCTURE ONLY.

These are the plain definitions the randomized method must reproduce in
expectation (and exactly at eps = 0), used to pin the C oracle on small graphs:

* Eq. (1) of the paper truncated at level L: pi_L = sum_{i<=L} w_i P^i x with
  P = D^-a A D^-b, evaluated by Horner's rule (dense, and with a sparse P for
  the error of full-size runs against the exact sum);
* PPR: pi = alpha (I - (1 - alpha) A D^-1)^-1 x (Section 2);
* single-target PPR: pi = alpha (I - (1 - alpha) D^-1 A)^-1 e_t (Section 2);
* Katz: pi = sum_i beta^i A^i x = (I - beta A)^-1 x for beta < 1/lambda_1;
* heat kernel PageRank: pi = e^{-t (I - A D^-1)} x (the series of Section 2);
* L-hop transition probability: (A D^-1)^L x (Section 1).
"""
from __future__ import annotations

import numpy as np


def adjacency(g) -> np.ndarray:
    A = np.zeros((g.n, g.n))
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    A[rows, g.col] = 1.0
    return A


def transition(g, a: float, b: float) -> np.ndarray:
    """P = D^-a A D^-b (isolated nodes get a zero row and column)."""
    A = adjacency(g)
    d = A.sum(axis=1)
    with np.errstate(divide="ignore"):
        da = np.where(d > 0, d ** (-a), 0.0)
        db = np.where(d > 0, d ** (-b), 0.0)
    return da[:, None] * A * db[None, :]


def horner(g, a: float, b: float, w, x) -> np.ndarray:
    """sum_{i=0}^{L} w_i P^i x for x of shape (n,) or (n, C)."""
    P = transition(g, a, b)
    w = np.asarray(w, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    acc = w[-1] * x
    for i in range(w.size - 2, -1, -1):
        acc = w[i] * x + P @ acc
    return acc


def transition_directed(g, a: float, b: float, reverse: bool = False) -> np.ndarray:
    """P = D^-a A~ D^-b of a directed graph given by its out-adjacency
    (Section 4, propagation on directed graphs): A~ = A^T pushes along
    out-edges, A~ = A (reverse) along in-edges; D holds the out-degrees, a
    node without out-arcs counting as out-degree 1."""
    A = adjacency(g)  # A[u, v] = 1 for the arc u -> v
    d = np.maximum(A.sum(axis=1), 1.0)
    At = A if reverse else A.T
    return (d ** (-a))[:, None] * At * (d ** (-b))[None, :]


def horner_directed(g, a: float, b: float, w, x, reverse: bool = False) -> np.ndarray:
    """sum_{i=0}^{L} w_i P^i x with the directed P of transition_directed."""
    P = transition_directed(g, a, b, reverse)
    w = np.asarray(w, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    acc = w[-1] * x
    for i in range(w.size - 2, -1, -1):
        acc = w[i] * x + P @ acc
    return acc


def horner_sparse(g, a: float, b: float, w, x) -> np.ndarray:
    """sum_{i=0}^{L} w_i P^i x as horner(), with P = D^-a A D^-b held as a
    scipy CSR matrix (for graphs too large for a dense n x n matrix)."""
    import scipy.sparse as sp

    n = g.n
    d = np.diff(np.asarray(g.row_ptr, dtype=np.int64)).astype(np.float64)
    with np.errstate(divide="ignore"):
        da = np.where(d > 0, d ** (-a), 0.0)
        db = np.where(d > 0, d ** (-b), 0.0)
    A = sp.csr_matrix((np.ones(len(g.col)), np.asarray(g.col), np.asarray(g.row_ptr)), shape=(n, n))
    P = sp.diags(da) @ A @ sp.diags(db)
    w = np.asarray(w, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    acc = w[-1] * x
    for i in range(w.size - 2, -1, -1):
        acc = w[i] * x + P @ acc
    return acc


def horner_sparse_directed(g, a: float, b: float, w, x, reverse: bool = False) -> np.ndarray:
    """horner_directed with a scipy CSR P (large directed graphs)."""
    import scipy.sparse as sp

    n = g.n
    rp = np.asarray(g.row_ptr, dtype=np.int64)
    A = sp.csr_matrix((np.ones(len(g.col)), np.asarray(g.col), rp), shape=(n, n))  # A[u, v]: u -> v
    d = np.maximum(np.diff(rp), 1).astype(np.float64)
    At = A if reverse else A.T
    P = sp.diags(d ** (-a)) @ At @ sp.diags(d ** (-b))
    w = np.asarray(w, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    acc = w[-1] * x
    for i in range(w.size - 2, -1, -1):
        acc = w[i] * x + P @ acc
    return acc


def level_norms(g, a: float, b: float, w, x) -> np.ndarray:
    """||Y_i P^i x||_1 for i = 0..L, with Y_i = sum_{k >= i} w_k (Definition 3.2)."""
    P = transition(g, a, b)
    w = np.asarray(w, dtype=np.float64)
    Y = np.cumsum(w[::-1])[::-1]
    v = np.asarray(x, dtype=np.float64)
    out = np.empty(w.size)
    for i in range(w.size):
        out[i] = Y[i] * np.abs(v).sum()
        v = P @ v
    return out


def ppr_inverse(g, alpha: float, x) -> np.ndarray:
    A = adjacency(g)
    d = A.sum(axis=0)
    AD = A / np.where(d > 0, d, 1.0)[None, :]
    return alpha * np.linalg.solve(np.eye(g.n) - (1.0 - alpha) * AD, np.asarray(x, float))


def single_target_ppr(g, alpha: float, t: int) -> np.ndarray:
    A = adjacency(g)
    d = A.sum(axis=1)
    DA = A / np.where(d > 0, d, 1.0)[:, None]
    e = np.zeros(g.n)
    e[t] = 1.0
    return alpha * np.linalg.solve(np.eye(g.n) - (1.0 - alpha) * DA, e)


def katz_inverse(g, beta: float, x) -> np.ndarray:
    A = adjacency(g)
    return np.linalg.solve(np.eye(g.n) - beta * A, np.asarray(x, float))


def hkpr_expm(g, t: float, x) -> np.ndarray:
    from scipy.linalg import expm

    A = adjacency(g)
    d = A.sum(axis=0)
    AD = A / np.where(d > 0, d, 1.0)[None, :]
    return expm(-t * (np.eye(g.n) - AD)) @ np.asarray(x, float)


def tp_power(g, L: int, x) -> np.ndarray:
    A = adjacency(g)
    d = A.sum(axis=0)
    AD = A / np.where(d > 0, d, 1.0)[None, :]
    return np.linalg.matrix_power(AD, L) @ np.asarray(x, float)


def lambda1(g) -> float:
    return float(np.linalg.eigvalsh(adjacency(g)).max())
