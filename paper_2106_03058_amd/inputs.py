"""Seeded synthetic inputs: graphs, signals, query sources and weight sequences.

This module produces *data* only. It holds none of the propagation method's
arithmetic (no residues, thresholds, sampling or sums), so both the HIP path and
the CPU oracle can be fed from it without sharing any code of the method.

Graphs are simple undirected graphs stored as CSR with every row sorted by
neighbour id and no duplicate entries (the problem statement of the paper,
Section 2, takes G undirected).  Stand-ins for the paper's datasets (Tables 3
and 4) are power-law graphs of the same shape:

* Chung-Lu graphs with expected degrees w_i ~ (i+1)^(-1/(gamma-1)), scaled to a
  mean degree and capped at sqrt(n * mean), endpoints drawn proportional to w.
* R-MAT graphs (Chakrabarti et al.) with quadrant probabilities (a, b, c, d).

Both are symmetrised, lose generator self-loops and duplicates, and may get
exactly one self-loop per node (the GNN convention of Section 2).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


@dataclass
class Graph:
    """Undirected simple graph in CSR form (rows sorted by neighbour id)."""

    n: int
    row_ptr: np.ndarray  # int64, n + 1
    col: np.ndarray  # int32, row_ptr[-1]

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    @property
    def degree(self) -> np.ndarray:
        return np.diff(self.row_ptr).astype(np.int64)

    def describe(self) -> dict:
        d = self.degree
        return {
            "n": self.n,
            "arcs": self.nnz,
            "mean_degree": float(d.mean()) if self.n else 0.0,
            "max_degree": int(d.max()) if self.n else 0,
            "isolated": int((d == 0).sum()),
        }


def csr_from_pairs(n: int, src: np.ndarray, dst: np.ndarray, *,
                   self_loops: bool = False) -> Graph:
    """Symmetrise (src, dst) pairs, drop loops and duplicates, build CSR.

    With ``self_loops`` one loop (u, u) is added to every row afterwards.
    """
    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int64)
    keep = src != dst
    src, dst = src[keep], dst[keep]
    key = np.concatenate([src * n + dst, dst * n + src])
    if self_loops:
        ids = np.arange(n, dtype=np.int64)
        key = np.concatenate([key, ids * n + ids])
    key = np.unique(key)
    rows = key // n
    col = (key - rows * n).astype(np.int32)
    counts = np.bincount(rows, minlength=n)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    return Graph(n, row_ptr, col)


def chung_lu(n: int, mean_degree: float, gamma: float, seed: int, *,
             pair_factor: float = 1.0, self_loops: bool = False) -> Graph:
    """Chung-Lu power-law graph; node 0 carries the largest expected degree.

    ``n * mean_degree / 2 * pair_factor`` endpoint pairs are drawn, each
    endpoint independently with probability proportional to its weight.
    ``pair_factor > 1`` offsets the pairs lost to loops and duplicates.
    """
    rng = np.random.default_rng(seed)
    w = (np.arange(n, dtype=np.float64) + 1.0) ** (-1.0 / (gamma - 1.0))
    w *= mean_degree * n / w.sum()
    np.minimum(w, math.sqrt(n * mean_degree), out=w)
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    m = int(round(n * mean_degree / 2.0 * pair_factor))
    src = np.empty(m, dtype=np.int64)
    dst = np.empty(m, dtype=np.int64)
    chunk = 1 << 24
    for lo in range(0, m, chunk):
        hi = min(m, lo + chunk)
        src[lo:hi] = np.searchsorted(cdf, rng.random(hi - lo), side="right")
        dst[lo:hi] = np.searchsorted(cdf, rng.random(hi - lo), side="right")
    np.minimum(src, n - 1, out=src)
    np.minimum(dst, n - 1, out=dst)
    return csr_from_pairs(n, src, dst, self_loops=self_loops)


def rmat(scale: int, edge_factor: int, a: float, b: float, c: float, seed: int,
         *, permute: bool = True, self_loops: bool = False, directed: bool = False) -> Graph:
    """R-MAT graph with 2^scale nodes and edge_factor * 2^scale generated edges.

    Node labels are shuffled by a seeded permutation so that hubs are not
    clustered at small ids.  directed: the arcs are kept as generated
    (out-adjacency, loops and duplicates dropped) instead of symmetrised.
    """
    rng = np.random.default_rng(seed)
    n = 1 << scale
    m = n * edge_factor
    t_a = np.uint32(min(int(a * 2**32), 2**32 - 1))
    t_ab = np.uint32(min(int((a + b) * 2**32), 2**32 - 1))
    t_abc = np.uint32(min(int((a + b + c) * 2**32), 2**32 - 1))
    src = np.zeros(m, dtype=np.int64)
    dst = np.zeros(m, dtype=np.int64)
    chunk = 1 << 24
    for lo in range(0, m, chunk):
        hi = min(m, lo + chunk)
        s = np.zeros(hi - lo, dtype=np.int64)
        d = np.zeros(hi - lo, dtype=np.int64)
        for _ in range(scale):
            u = rng.integers(0, 2**32, size=hi - lo, dtype=np.uint32)
            bit_src = u >= t_ab  # quadrants c and d
            bit_dst = ((u >= t_a) & (u < t_ab)) | (u >= t_abc)  # b and d
            s = (s << 1) | bit_src
            d = (d << 1) | bit_dst
        src[lo:hi] = s
        dst[lo:hi] = d
    if permute:
        perm = rng.permutation(n).astype(np.int64)
        src = perm[src]
        dst = perm[dst]
    if directed:  # arcs src -> dst as generated (out-adjacency)
        return directed_from_pairs(n, src, dst)
    return csr_from_pairs(n, src, dst, self_loops=self_loops)


def erdos_renyi(n: int, p: float, seed: int, *, self_loops: bool = False) -> Graph:
    """G(n, p) on a small node count (used for closed-form checks)."""
    rng = np.random.default_rng(seed)
    iu, ju = np.triu_indices(n, k=1)
    keep = rng.random(iu.size) < p
    return csr_from_pairs(n, iu[keep], ju[keep], self_loops=self_loops)


def directed_from_pairs(n: int, src: np.ndarray, dst: np.ndarray) -> Graph:
    """Out-adjacency CSR of the arcs src -> dst (loops and duplicates dropped,
    no symmetrisation): row u lists the out-neighbours of u."""
    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int64)
    keep = src != dst
    key = np.unique(src[keep] * n + dst[keep])
    rows = key // n
    col = (key - rows * n).astype(np.int32)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=n), out=row_ptr[1:])
    return Graph(n, row_ptr, col)


def directed_chung_lu(n: int, mean_degree: float, gamma: float, seed: int, *, pair_factor: float = 1.0) -> Graph:
    """Directed power-law graph: n * mean_degree * pair_factor arcs whose tail
    and head are drawn independently with probability proportional to the
    Chung-Lu weights (node 0 heaviest); some nodes end up without out-arcs."""
    rng = np.random.default_rng(seed)
    w = (np.arange(n, dtype=np.float64) + 1.0) ** (-1.0 / (gamma - 1.0))
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    m = int(round(n * mean_degree * pair_factor))
    src = np.minimum(np.searchsorted(cdf, rng.random(m), side="right"), n - 1)
    dst = np.minimum(np.searchsorted(cdf, rng.random(m), side="right"), n - 1)
    perm = rng.permutation(n)  # tails and heads get independent hub orders
    return directed_from_pairs(n, src, perm[dst])


def toy_graph(k: int) -> Graph:
    """The bad case for pruned propagation in Section 4 (Figure 1).

    Node 0 is s, nodes 1..k are u_1..u_k and node k+1 is v; every u_i is joined
    to s and to v.  A 2-step walk from s ends at s or v with probability 1/2
    each and never at a u_i.
    """
    u = np.arange(1, k + 1, dtype=np.int64)
    src = np.concatenate([np.zeros(k, dtype=np.int64), u])
    dst = np.concatenate([u, np.full(k, k + 1, dtype=np.int64)])
    return csr_from_pairs(k + 2, src, dst)


def path_graph(n: int) -> Graph:
    i = np.arange(n - 1, dtype=np.int64)
    return csr_from_pairs(n, i, i + 1)


def star_graph(k: int) -> Graph:
    return csr_from_pairs(k + 1, np.zeros(k, dtype=np.int64),
                          np.arange(1, k + 1, dtype=np.int64))


# ----------------------------------------------------------------- signals

def one_hot(n: int, sources, dtype=np.float32) -> np.ndarray:
    """n x C matrix whose column c is the indicator of node sources[c]."""
    sources = np.asarray(sources, dtype=np.int64)
    x = np.zeros((n, sources.size), dtype=dtype)
    x[sources, np.arange(sources.size)] = 1
    return x


def features_normal(n: int, cols: int, seed: int) -> np.ndarray:
    """n x cols float32 matrix with i.i.d. N(0, 1) entries."""
    return np.random.default_rng(seed).standard_normal((n, cols), dtype=np.float32)


def features_uniform(n: int, cols: int, lo: float, hi: float, seed: int) -> np.ndarray:
    """n x cols float32 matrix with i.i.d. U[lo, hi) entries."""
    r = np.random.default_rng(seed).random((n, cols), dtype=np.float32)
    return (lo + (hi - lo) * r).astype(np.float32)


def sources_uniform(g: Graph, k: int, seed: int) -> np.ndarray:
    """k distinct-when-possible sources, uniform over nodes with degree >= 1."""
    rng = np.random.default_rng(seed)
    cand = np.flatnonzero(g.degree >= 1)
    return rng.choice(cand, size=k, replace=k > cand.size).astype(np.int64)


def sources_by_degree(g: Graph, k: int, seed: int) -> np.ndarray:
    """k sources drawn with probability proportional to degree."""
    rng = np.random.default_rng(seed)
    d = g.degree.astype(np.float64)
    return rng.choice(g.n, size=k, p=d / d.sum()).astype(np.int64)


# ------------------------------------------------- weight sequences (Table 1)

def weights_ppr(alpha: float, L: int) -> np.ndarray:
    """w_i = alpha (1 - alpha)^i, i = 0..L (PageRank / PPR / APPNP)."""
    w = np.empty(L + 1)
    v = alpha
    for i in range(L + 1):
        w[i] = v
        v *= 1.0 - alpha
    return w


def weights_hkpr(t: float, L: int) -> np.ndarray:
    """w_i = e^-t t^i / i!, i = 0..L (heat kernel PageRank / GDC)."""
    w = np.empty(L + 1)
    v = math.exp(-t)
    for i in range(L + 1):
        w[i] = v
        v = v * t / (i + 1)
    return w


def weights_katz(beta: float, L: int, scale: float = 1.0) -> np.ndarray:
    """w_i = scale * beta^i, i = 0..L (Katz)."""
    w = np.empty(L + 1)
    v = scale
    for i in range(L + 1):
        w[i] = v
        v *= beta
    return w


def weights_tp(L: int) -> np.ndarray:
    """w_L = 1 and w_i = 0 otherwise (L-hop transition probability)."""
    w = np.zeros(L + 1)
    w[L] = 1.0
    return w


def lambda_max(g: Graph, *, tol: float = 1e-10, max_iter: int = 1000) -> float:
    """Largest adjacency eigenvalue by FP64 power iteration from all-ones.

    Stops when the Rayleigh estimate changes by less than ``tol`` relative.
    """
    import scipy.sparse as sp

    a = sp.csr_matrix((np.ones(g.nnz), g.col, g.row_ptr), shape=(g.n, g.n))
    v = np.ones(g.n)
    v /= np.linalg.norm(v)
    lam = 0.0
    for _ in range(max_iter):
        y = a @ v
        new = float(v @ y)
        nrm = np.linalg.norm(y)
        if nrm == 0.0:
            return 0.0
        v = y / nrm
        if lam and abs(new - lam) <= tol * abs(new):
            return new
        lam = new
    return lam


# ------------------------------------------------ device-side generation
# Large stand-ins (hundreds of millions of arcs) are generated with PyTorch on
# the GPU: the same recipes as above, seeded, returning CSR tensors on the
# device (and nothing of the propagation method).

def rmat_device(scale: int, edge_factor: int, a: float, b: float, c: float, seed: int,
                device="cuda:0", chunk: int = 1 << 26):
    """R-MAT graph built on the GPU; returns (n, row_ptr int64, col int32) tensors.

    Quadrants from uniform floats per bit level, labels shuffled by a seeded
    permutation, symmetrised, loops dropped, duplicates removed."""
    import torch

    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    n = 1 << scale
    m = n * edge_factor
    keys = []
    perm = torch.randperm(n, generator=gen, device=device)
    for lo in range(0, m, chunk):
        k = min(chunk, m - lo)
        s = torch.zeros(k, dtype=torch.int64, device=device)
        d = torch.zeros(k, dtype=torch.int64, device=device)
        for _ in range(scale):
            u = torch.rand(k, generator=gen, device=device, dtype=torch.float64)
            bs = u >= (a + b)
            bd = ((u >= a) & (u < a + b)) | (u >= a + b + c)
            s = s * 2 + bs.to(torch.int64)
            d = d * 2 + bd.to(torch.int64)
        s = perm[s]
        d = perm[d]
        keep = s != d
        s, d = s[keep], d[keep]
        keys.append(s * n + d)
        keys.append(d * n + s)
        del s, d, keep
    key = torch.unique(torch.cat(keys))
    del keys
    rows = torch.div(key, n, rounding_mode="floor")
    col = (key - rows * n).to(torch.int32)
    counts = torch.bincount(rows, minlength=n)
    row_ptr = torch.zeros(n + 1, dtype=torch.int64, device=device)
    row_ptr[1:] = torch.cumsum(counts, 0)
    return n, row_ptr, col


def chung_lu_device(n: int, mean_degree: float, gamma: float, seed: int, *, target_edges: int | None = None,
                    pair_factor: float = 1.0, device="cuda:0", chunk: int = 1 << 26, max_rounds: int = 4):
    """Chung-Lu power-law graph built on the GPU with the recipe of chung_lu
    (weights (i+1)^(-1/(gamma-1)) scaled to the mean degree and capped at
    sqrt(n mean_degree), endpoints drawn proportionally to weight by inverse
    CDF); loops dropped, duplicates removed, symmetrised.  With target_edges,
    more pairs are drawn (same generator) until that many distinct undirected
    edges exist, making up for the pairs lost to loops and duplicates.
    Returns (n, row_ptr int64, col int32) tensors."""
    import torch

    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    # the weights and their CDF on the host: a device scan may add in an
    # order that changes from run to run, and with it the sampled graph
    w = (np.arange(n, dtype=np.float64) + 1.0) ** (-1.0 / (gamma - 1.0))
    w *= mean_degree * n / float(w.sum())
    np.minimum(w, math.sqrt(n * mean_degree), out=w)
    cdf = np.cumsum(w)
    del w
    cdf /= cdf[-1]
    cdf = torch.from_numpy(cdf).to(device)

    def draw(m):
        keys = []
        for lo in range(0, m, chunk):
            k = min(chunk, m - lo)
            s = torch.searchsorted(cdf, torch.rand(k, generator=gen, device=device, dtype=torch.float64),
                                   right=True).clamp_(max=n - 1)
            d = torch.searchsorted(cdf, torch.rand(k, generator=gen, device=device, dtype=torch.float64),
                                   right=True).clamp_(max=n - 1)
            keep = s != d
            s, d = s[keep], d[keep]
            keys.append(torch.minimum(s, d) * n + torch.maximum(s, d))
            del s, d, keep
        return torch.unique(torch.cat(keys))

    m = int(round(n * mean_degree / 2.0 * pair_factor))
    key = draw(m)
    for _ in range(max_rounds):
        if target_edges is None or key.numel() >= target_edges:
            break
        short = target_edges - key.numel()
        lost = 1.0 - key.numel() / float(m)  # fraction of drawn pairs lost so far
        extra = int(short / max(1.0 - 2.0 * lost, 0.25) * 1.02) + 1
        m += extra
        key = torch.unique(torch.cat([key, draw(extra)]))
    del cdf
    u = torch.div(key, n, rounding_mode="floor")
    v = key - u * n
    del key
    both = torch.cat([u * n + v, v * n + u])
    del u, v
    both, _ = torch.sort(both)
    rows = torch.div(both, n, rounding_mode="floor")
    col = (both - rows * n).to(torch.int32)
    del both
    counts = torch.bincount(rows, minlength=n)
    del rows
    row_ptr = torch.zeros(n + 1, dtype=torch.int64, device=device)
    row_ptr[1:] = torch.cumsum(counts, 0)
    return n, row_ptr, col


def add_self_loops(n: int, row_ptr: np.ndarray, col: np.ndarray) -> Graph:
    """The CSR graph with one loop (u, u) appended to every row (GNN
    propagation on A + I)."""
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    deg = np.diff(row_ptr)
    new_rp = row_ptr + np.arange(n + 1, dtype=np.int64)
    new_col = np.empty(int(new_rp[-1]), dtype=np.int32)
    shift = np.repeat(np.arange(n, dtype=np.int64), deg)  # entries of row u move by u
    new_col[np.arange(col.size, dtype=np.int64) + shift] = col
    del shift
    new_col[new_rp[1:] - 1] = np.arange(n, dtype=np.int32)
    return Graph(n, new_rp, new_col)


def add_self_loops_device(n: int, row_ptr, col, chunk: int = 1 << 27):
    """add_self_loops on device tensors (int64 row_ptr, int32 col): returns
    the (row_ptr, col) tensors of the CSR with one loop appended to every row."""
    import torch

    dev = row_ptr.device
    new_rp = row_ptr + torch.arange(n + 1, device=dev, dtype=torch.int64)
    new_col = torch.empty(int(new_rp[-1].item()), dtype=torch.int32, device=dev)
    nnz = col.numel()
    for lo in range(0, nnz, chunk):  # entry k of row u moves to k + u
        k = torch.arange(lo, min(lo + chunk, nnz), device=dev, dtype=torch.int64)
        u = torch.searchsorted(row_ptr, k, right=True) - 1
        new_col[k + u] = col[lo:lo + k.numel()]
        del k, u
    new_col[new_rp[1:] - 1] = torch.arange(n, device=dev, dtype=torch.int32)
    return new_rp, new_col


def features_uniform_device(n: int, C: int, lo: float, hi: float, seed: int, device="cuda:0"):
    """n x C binary32 features, i.i.d. uniform on [lo, hi), generated on the GPU."""
    import torch

    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    x = torch.rand((n, C), generator=gen, device=device, dtype=torch.float32)
    x.mul_(hi - lo).add_(lo)
    return x


def lambda_max_device(n: int, row_ptr, col, *, tol: float = 1e-10, max_iter: int = 1000) -> float:
    """Largest adjacency eigenvalue by FP64 power iteration on the GPU."""
    import torch

    vals = torch.ones(col.numel(), dtype=torch.float64, device=col.device)
    A = torch.sparse_csr_tensor(row_ptr, col.to(torch.int64), vals, size=(n, n))
    v = torch.full((n, 1), 1.0 / float(n) ** 0.5, dtype=torch.float64, device=col.device)
    lam = 0.0
    for _ in range(max_iter):
        y = A @ v
        new = float((v * y).sum())
        nrm = float(torch.linalg.vector_norm(y))
        if nrm == 0.0:
            return 0.0
        v = y / nrm
        if lam and abs(new - lam) <= tol * abs(new):
            return new
        lam = new
    return lam
