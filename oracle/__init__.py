"""CPU oracle for randomized graph propagation -- TEST INFRASTRUCTURE ONLY.

A plain sequential reference of Algorithm 2 (Section 4 of "Approximate Graph
Propagation", KDD'21) written in C (``agp_oracle.c``) plus dense FP64 closed
forms (``dense.py``).  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package; the product library
never calls it and shares no code with it.
"""
from __future__ import annotations

import ctypes as ct
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "agp_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no FMA contraction, IEEE binary64)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.run(
            ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-ffp-contract=off", "-fno-fast-math",
             "-fPIC", "-shared", "-pthread", _SRC, "-o", tmp, "-lm"],
            check=True)
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = ct.CDLL(_LIB)
        i64p = ct.POINTER(ct.c_int64)
        i32p = ct.POINTER(ct.c_int32)
        u32p = ct.POINTER(ct.c_uint32)
        u64p = ct.POINTER(ct.c_uint64)
        dp = ct.POINTER(ct.c_double)
        L.orc_sweep.argtypes = [ct.c_int64, i64p, i32p, dp, i32p, ct.POINTER(ct.c_int64), ct.POINTER(ct.c_double)]
        L.orc_degree_sort.argtypes = [ct.c_int64, i64p, i32p, i32p, i32p, i32p, i32p, ct.c_int32]
        L.orc_level_tables.argtypes = [dp, ct.c_int32, ct.c_int32, dp, dp, dp, dp]
        L.orc_theta.argtypes = [dp, ct.c_int64, ct.c_double]
        L.orc_theta.restype = ct.c_double
        L.orc_philox4x32_10.argtypes = [u32p, u32p, u32p]
        L.orc_skip.argtypes = [ct.c_double, ct.c_double]
        L.orc_skip.restype = ct.c_int32
        L.orc_splitmix64.argtypes = [ct.c_uint64]
        L.orc_splitmix64.restype = ct.c_uint64
        L.orc_exact_sum.argtypes = [dp, ct.c_int64, ct.c_int32]
        L.orc_exact_sum.restype = ct.c_double
        L.orc_propagate_many.argtypes = [ct.c_int64, i64p, i32p, i32p, ct.c_double, ct.c_double,
                                         dp, ct.c_int32, ct.c_int32, dp, ct.c_int32, ct.c_double, ct.c_uint64,
                                         u32p, ct.c_int32, dp, u64p, ct.c_int32, ct.c_int32, ct.c_int32]
        L.orc_exact_sum_horner.argtypes = [ct.c_int64, i64p, i32p, i32p, ct.c_double, ct.c_double, dp,
                                           ct.c_int32, dp, ct.c_int32, dp, ct.c_int32, ct.c_int32]
        _lib = L
    return _lib


def _p(a, t):
    return a.ctypes.data_as(ct.POINTER(t))


@dataclass
class SortedGraph:
    """Graph whose adjacency lists are sorted by (neighbour factor degree, id).

    deg: row lengths; fdeg: the degrees in the factors d^-a, d^-b (row
    lengths of an undirected graph, out-degrees of a directed one; >= 1)."""

    n: int
    row_ptr: np.ndarray
    col: np.ndarray
    deg: np.ndarray
    fdeg: np.ndarray


def degree_sort(g, fdeg=None, threads: int | None = None) -> SortedGraph:
    """Adjacency lists sorted by (neighbour factor degree, id) (Section 4);
    rows are sorted by `threads` host threads (default: all cores, at most 16)."""
    rp = np.ascontiguousarray(g.row_ptr, dtype=np.int64)
    col = np.ascontiguousarray(g.col, dtype=np.int32)
    out = np.empty_like(col)
    deg = np.empty(g.n, dtype=np.int32)
    fd = np.empty(g.n, dtype=np.int32)
    fin = None if fdeg is None else np.ascontiguousarray(fdeg, dtype=np.int32)
    rc = lib().orc_degree_sort(g.n, _p(rp, ct.c_int64), _p(col, ct.c_int32),
                               None if fin is None else _p(fin, ct.c_int32),
                               _p(out, ct.c_int32), _p(deg, ct.c_int32), _p(fd, ct.c_int32),
                               int(threads or min(16, os.cpu_count() or 1)))
    assert rc == 0
    return SortedGraph(g.n, rp, out, deg, fd)


def directed(g, reverse: bool = False) -> SortedGraph:
    """A directed graph given by its out-adjacency CSR (Section 4, propagation
    on directed graphs): pushes follow out-edges (A~ = A^T), or in-edges when
    reverse (A~ = A, single-target proximity); the factors use out-degrees."""
    rp = np.asarray(g.row_ptr, dtype=np.int64)
    outdeg = np.diff(rp).astype(np.int32)
    if not reverse:
        return degree_sort(g, outdeg)
    src = np.repeat(np.arange(g.n, dtype=np.int64), np.diff(rp))
    dst = np.asarray(g.col, dtype=np.int64)
    order = np.lexsort((src, dst))  # rows of the transpose: in-neighbours of each node
    trp = np.zeros(g.n + 1, dtype=np.int64)
    np.cumsum(np.bincount(dst, minlength=g.n), out=trp[1:])
    gt = type(g)(g.n, trp, src[order].astype(np.int32))
    return degree_sort(gt, outdeg)


def level_tables(w, tail: bool = False):
    """S, Y_0..Y_{L+1}, rho, kappa (tail: the infinite-tail reading of Y_i)."""
    w = np.ascontiguousarray(w, dtype=np.float64)
    L = w.size - 1
    S = ct.c_double()
    Y = np.empty(L + 2)
    rho = np.empty(L + 1)
    kappa = np.empty(L + 1)
    rc = lib().orc_level_tables(_p(w, ct.c_double), L, int(bool(tail)), ct.byref(S), _p(Y, ct.c_double),
                                _p(rho, ct.c_double), _p(kappa, ct.c_double))
    if rc != 0:
        raise ValueError("weights rejected")
    return S.value, Y, rho, kappa


def theta(x, eps: float) -> float:
    x = np.ascontiguousarray(x, dtype=np.float64)
    return lib().orc_theta(_p(x, ct.c_double), x.size, eps)


def philox(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    o = np.empty(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_p(c, ct.c_uint32), _p(k, ct.c_uint32), _p(o, ct.c_uint32))
    return o


def skip(p: float, V: float) -> int:
    return lib().orc_skip(p, V)


def splitmix64(x: int) -> int:
    return lib().orc_splitmix64(x)


def exact_sum(vals, wp: int) -> float:
    v = np.ascontiguousarray(vals, dtype=np.float64)
    return lib().orc_exact_sum(_p(v, ct.c_double), v.size, wp)


COUNTER_NAMES = ("frontier", "hash", "det", "cand", "acc", "runs")


SPLIT_QID_BIT = 1 << 23


def propagate(sg: SortedGraph, a: float, b: float, w, x, eps: float, seed: int, *,
              wp: int = 32, qids=None, threads: int | None = None, tail: bool = False,
              split_signs: bool = False, stop_level: int = -1, sample_stride: int = 1):
    """Run Algorithm 2 on every column of x (n x C, or a length-n vector).

    Returns (out, counters): out has the shape of x (float64 values that are
    binary32 values when wp == 32); counters maps each counter name to a
    C x (L + 1) uint64 array.

    tail: the paper-literal Y_i = 1 - sum_{k<i} w_k (weights summing to at
    most 1, no rescaling), see orc_level_tables.

    stop_level: stop after that level (a bounded timing sample: the output
    then holds the reserves of the levels done, the counters of those
    levels are complete).  sample_stride: at the stop level, visit only the
    nodes whose id is a multiple of it (a smaller timing sample).

    split_signs: the literal treatment of signed signals (Section 3,
    assumption on the graph signal): x+ (the positive entries) and x- (the
    negative ones) are propagated as separate signals, each with its own
    threshold eps * ||x+-||_1, column c's x- part drawing from the random
    stream of query id qid_c + 2^23; the estimate is pi+ + pi- rounded once to
    the working precision, and the counters are those of both passes added.
    """
    if split_signs:
        X = np.asarray(x, dtype=np.float64).reshape(sg.n, -1)
        C = X.shape[1]
        q = np.arange(C, dtype=np.uint32) if qids is None else np.ascontiguousarray(qids, dtype=np.uint32)
        if q.size != C or (q >= SPLIT_QID_BIT).any():
            raise ValueError("split_signs needs one qid per column, each below 2^23")
        xp = np.where(X > 0.0, X, 0.0)
        xn = np.where(X < 0.0, X, 0.0)
        op, cp = propagate(sg, a, b, w, xp, eps, seed, wp=wp, qids=q, threads=threads, tail=tail)
        on, cn = propagate(sg, a, b, w, xn, eps, seed, wp=wp, qids=q + np.uint32(SPLIT_QID_BIT), threads=threads,
                           tail=tail)
        if wp == 32:
            res = (op.astype(np.float32) + on.astype(np.float32)).astype(np.float64)
        else:
            res = op + on
        counters = {k: cp[k] + cn[k] for k in cp}
        return (res[:, 0].copy() if np.asarray(x).ndim == 1 else res), counters
    w = np.ascontiguousarray(w, dtype=np.float64)
    L = w.size - 1
    x = np.asarray(x)
    vec = x.ndim == 1
    X = x.reshape(sg.n, -1)
    C = X.shape[1]
    xc = np.ascontiguousarray(X.T, dtype=np.float64)  # column-major
    out = np.empty_like(xc)
    cnt = np.zeros((C, len(COUNTER_NAMES), L + 1), dtype=np.uint64)
    q = None if qids is None else np.ascontiguousarray(qids, dtype=np.uint32)
    if threads is None:
        threads = min(C, os.cpu_count() or 1)
    rc = lib().orc_propagate_many(
        sg.n, _p(sg.row_ptr, ct.c_int64), _p(sg.col, ct.c_int32), _p(sg.fdeg, ct.c_int32),
        float(a), float(b), _p(w, ct.c_double), L, int(bool(tail)), _p(xc, ct.c_double), C, float(eps),
        ct.c_uint64(seed & 0xFFFFFFFFFFFFFFFF), None if q is None else _p(q, ct.c_uint32), wp,
        _p(out, ct.c_double), _p(cnt, ct.c_uint64), max(1, int(threads)), int(stop_level), int(sample_stride))
    if rc != 0:
        raise ValueError("oracle rejected the arguments")
    res = out.T
    counters = {name: cnt[:, k, :] for k, name in enumerate(COUNTER_NAMES)}
    return (res[:, 0].copy() if vec else np.ascontiguousarray(res)), counters


def sweep(g, pi):
    """Local clustering sweep of Section 5 on the estimate pi (length n):
    returns (best_size, best_conductance, order); the cluster is
    order[:best_size]."""
    rp = np.ascontiguousarray(g.row_ptr, dtype=np.int64)
    col = np.ascontiguousarray(g.col, dtype=np.int32)
    p = np.ascontiguousarray(pi, dtype=np.float64)
    order = np.empty(g.n, dtype=np.int32)
    size = ct.c_int64()
    phi = ct.c_double()
    rc = lib().orc_sweep(g.n, _p(rp, ct.c_int64), _p(col, ct.c_int32), _p(p, ct.c_double), _p(order, ct.c_int32),
                         ct.byref(size), ct.byref(phi))
    assert rc == 0
    return size.value, phi.value, order


def truncated_sum(g, a: float, b: float, w, x, *, fdeg=None, threads: int | None = None,
                  verbose: bool = False) -> np.ndarray:
    """Eq. 1 truncated at L in binary64, without sampling or thresholds:
    sum_{i=0..L} w_i (D^-a A D^-b)^i x by Horner's rule (orc_exact_sum_horner),
    with row v of g listing the nodes that push into v (the CSR itself for an
    undirected graph).  x: n x C (C <= 64) or a vector; threads share rows."""
    w = np.ascontiguousarray(w, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    vec = x.ndim == 1
    X = np.ascontiguousarray(x.reshape(g.n, -1))
    C = X.shape[1]
    out = np.empty_like(X)
    rp = np.ascontiguousarray(g.row_ptr, dtype=np.int64)
    col = np.ascontiguousarray(g.col, dtype=np.int32)
    fd = None if fdeg is None else np.ascontiguousarray(fdeg, dtype=np.int32)
    rc = lib().orc_exact_sum_horner(g.n, _p(rp, ct.c_int64), _p(col, ct.c_int32),
                                    None if fd is None else _p(fd, ct.c_int32), float(a), float(b),
                                    _p(w, ct.c_double), w.size - 1, _p(X, ct.c_double), C, _p(out, ct.c_double),
                                    int(threads or min(16, os.cpu_count() or 1)), int(bool(verbose)))
    if rc != 0:
        raise ValueError("oracle rejected the arguments")
    return out[:, 0].copy() if vec else out
