"""Python binding of libagp: argument marshalling only.

Every step of the propagation runs in the HIP kernels behind the C ABI of
``include/agp.h``; PyTorch is used for device memory and streams.  Importing
this module does not need a GPU, but every call does, and a missing
``libagp.so`` is an error (there is no fallback path).
"""
from __future__ import annotations

import ctypes as ct
import os
import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libagp.so")

AGP_OK, AGP_EINVAL, AGP_ENOMEM, AGP_EDEVICE, AGP_ERANGE, AGP_ENOTSUP = 0, 1, 2, 3, 4, 5
AGP_PENDING, AGP_ENOENT, AGP_EBUSY = 6, 7, 8
AGP_HOST_PTRS, AGP_VALIDATE, AGP_ADD_SELF_LOOPS, AGP_DIRECTED, AGP_REVERSE = 1, 2, 4, 8, 16
MAX_LEVELS = 255

EXPORTED = [
    "agp_last_error", "agp_graph_create", "agp_graph_info", "agp_graph_export",
    "agp_graph_destroy", "agp_propagate", "agp_propagate_f64", "agp_weights_ppr",
    "agp_weights_hkpr", "agp_weights_katz", "agp_weights_tp", "agp_server_create", "agp_submit",
    "agp_poll", "agp_server_destroy", "agp_autotune", "agp_get_tuning", "agp_sweep",
    "agp_propagate_variant", "agp_propagate_variant_f64", "agp_sweep_batch", "agp_graph_groups",
    "agp_device_philox4x32_10", "agp_device_splitmix64", "agp_set_tuning", "agp_propagate_noalloc",
]
NOALLOC_SCRATCH_BYTES = 64 << 20
AGP_VARIANT_INFINITE_TAIL, AGP_VARIANT_SPLIT_SIGNS = 1, 2


class AGPError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[{code}] {msg}")
        self.code = code


class Stats(ct.Structure):
    _fields_ = [
        ("levels", ct.c_int32), ("columns", ct.c_int32), ("tiles", ct.c_int32), ("dense", ct.c_int32),
        ("frontier", ct.c_uint64 * (MAX_LEVELS + 1)),
        ("hash", ct.c_uint64 * (MAX_LEVELS + 1)),
        ("det", ct.c_uint64 * (MAX_LEVELS + 1)),
        ("cand", ct.c_uint64 * (MAX_LEVELS + 1)),
        ("acc", ct.c_uint64 * (MAX_LEVELS + 1)),
        ("runs", ct.c_uint64 * (MAX_LEVELS + 1)),
        ("device_ms", ct.c_double),
        ("level_ms", ct.c_double * (MAX_LEVELS + 1)),
        ("level_total_ms", ct.c_double * (MAX_LEVELS + 1)),
    ]

    def to_dict(self) -> dict:
        L = self.levels
        d = {k: np.array(getattr(self, k)[: L + 1], dtype=np.uint64)
             for k in ("frontier", "hash", "det", "cand", "acc", "runs")}
        d["levels"] = L
        d["columns"] = self.columns
        d["tiles"] = self.tiles
        d["dense"] = bool(self.dense)
        d["device_ms"] = float(self.device_ms)
        d["level_ms"] = np.array(self.level_ms[: L + 1], dtype=np.float64)
        d["level_total_ms"] = np.array(self.level_total_ms[: L + 1], dtype=np.float64)
        d["pushes"] = int(d["det"].sum() + d["acc"].sum())
        return d


_lib = None


def lib():
    """Load libagp.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = ct.CDLL(LIB_PATH)
        vp, dp = ct.c_void_p, ct.POINTER(ct.c_double)
        i64p, i32p, u32p = ct.POINTER(ct.c_int64), ct.POINTER(ct.c_int32), ct.POINTER(ct.c_uint32)
        L.agp_last_error.restype = ct.c_char_p
        L.agp_graph_create.argtypes = [ct.c_int64, ct.c_int64, vp, vp, ct.c_uint32, vp, ct.POINTER(vp)]
        L.agp_graph_info.argtypes = [vp, i64p, i64p, i32p]
        L.agp_graph_export.argtypes = [vp, i64p, i32p, i32p]
        L.agp_graph_groups.argtypes = [vp, ct.POINTER(ct.c_uint8)]
        L.agp_graph_destroy.argtypes = [vp]
        prop = [vp, ct.c_double, ct.c_double, dp, ct.c_int32, vp, ct.c_int32, ct.c_double,
                ct.c_uint64, u32p, vp, vp, ct.POINTER(Stats)]
        L.agp_propagate.argtypes = prop
        L.agp_propagate_f64.argtypes = prop
        var = prop[:10] + [ct.c_uint32] + prop[10:]
        L.agp_propagate_noalloc.argtypes = prop[:-1]
        L.agp_propagate_variant.argtypes = var
        L.agp_propagate_variant_f64.argtypes = var
        L.agp_weights_ppr.argtypes = [ct.c_double, ct.c_int32, dp]
        L.agp_weights_hkpr.argtypes = [ct.c_double, ct.c_int32, dp]
        L.agp_weights_katz.argtypes = [ct.c_double, ct.c_int32, dp]
        L.agp_weights_tp.argtypes = [ct.c_int32, dp]
        L.agp_sweep.argtypes = [vp, vp, ct.c_int64, vp, i64p, dp, vp]
        L.agp_sweep_batch.argtypes = [vp, vp, ct.c_int64, ct.c_int32, vp, i64p, dp]
        L.agp_device_philox4x32_10.argtypes = [ct.c_int64, vp, vp, vp]
        L.agp_device_splitmix64.argtypes = [ct.c_int64, vp, vp]
        _lib = L
    return _lib


def _check(rc: int) -> None:
    if rc != AGP_OK:
        raise AGPError(rc, lib().agp_last_error().decode(errors="replace"))


def _stream_ptr(stream) -> int:
    import torch

    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _dptr(t) -> int:
    return int(t.data_ptr())


class Graph:
    """A graph resident on the GPU with degree-sorted adjacency lists."""

    def __init__(self, row_ptr, col, *, validate: bool = False, self_loops: bool = False,
                 directed: bool = False, reverse: bool = False, stream=None):
        """row_ptr / col: host arrays, or CUDA tensors (int64 / int32) on the device.

        directed: rows are out-neighbour lists of a directed graph and pushes
        follow out-edges; reverse (with directed): pushes follow in-edges."""
        flags = ((AGP_VALIDATE if validate else 0) | (AGP_ADD_SELF_LOOPS if self_loops else 0) |
                 (AGP_DIRECTED if directed else 0) | (AGP_REVERSE if reverse else 0))
        if hasattr(row_ptr, "is_cuda") and row_ptr.is_cuda:
            import torch

            if row_ptr.dtype != torch.int64 or col.dtype != torch.int32:
                raise ValueError("device CSR needs int64 row_ptr and int32 col")
            rp_t, cl_t = row_ptr.contiguous(), col.contiguous()
            n = rp_t.numel() - 1
            nnz = int(rp_t[-1].item())
            rp_p, cl_p = rp_t.data_ptr(), (cl_t.data_ptr() if cl_t.numel() else None)
        else:
            rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
            cl = np.ascontiguousarray(col, dtype=np.int32)
            n = rp.size - 1
            nnz = int(rp[-1])
            flags |= AGP_HOST_PTRS
            rp_p, cl_p = rp.ctypes.data, (cl.ctypes.data if cl.size else None)
        h = ct.c_void_p()
        _check(lib().agp_graph_create(n, nnz, rp_p, cl_p, flags, _stream_ptr(stream), ct.byref(h)))
        self._h = h
        n_, nnz, md = ct.c_int64(), ct.c_int64(), ct.c_int32()
        _check(lib().agp_graph_info(h, ct.byref(n_), ct.byref(nnz), ct.byref(md)))
        self.n, self.nnz, self.max_degree = n_.value, nnz.value, md.value

    @classmethod
    def from_inputs(cls, g, **kw) -> "Graph":
        return cls(g.row_ptr, g.col, **kw)

    @property
    def handle(self):
        if self._h is None:
            raise RuntimeError("graph was destroyed")
        return self._h

    def export(self):
        rp = np.empty(self.n + 1, dtype=np.int64)
        col = np.empty(self.nnz, dtype=np.int32)
        deg = np.empty(self.n, dtype=np.int32)
        _check(lib().agp_graph_export(self.handle, rp.ctypes.data_as(ct.POINTER(ct.c_int64)),
                                      col.ctypes.data_as(ct.POINTER(ct.c_int32)),
                                      deg.ctypes.data_as(ct.POINTER(ct.c_int32))))
        return rp, col, deg

    def groups(self) -> np.ndarray:
        """Degree group floor(log2 d) of every arc's neighbour, in export() order."""
        gid = np.empty(self.nnz, dtype=np.uint8)
        _check(lib().agp_graph_groups(self.handle, gid.ctypes.data_as(ct.POINTER(ct.c_uint8))))
        return gid

    def close(self) -> None:
        if getattr(self, "_h", None) is not None:
            lib().agp_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def propagate(graph: Graph, a: float, b: float, w, x, eps: float, seed: int, *, qids=None,
              out=None, stream=None, stats: bool = False, tail: bool = False, split_signs: bool = False):
    """Run the randomized propagation on every column of x.

    x: CUDA tensor (n,) or (n, C), float32 (binary32 path) or float64.
    Returns (out, stats) where out has the shape and dtype of x and stats is
    a dict of per-level counters (or None).  tail / split_signs select the
    paper-literal variants (agp_propagate_variant).
    """
    import torch

    if not x.is_cuda:
        raise ValueError("x must be a device tensor")
    vec = x.dim() == 1
    X = x.reshape(graph.n, -1)
    if not X.is_contiguous():
        X = X.contiguous()
    C = X.shape[1]
    if out is None:
        out = torch.empty_like(X)
    o = out.reshape(graph.n, -1)
    if not o.is_contiguous() or o.dtype != X.dtype or o.shape != X.shape:
        raise ValueError("out must be a contiguous tensor of x's shape and dtype")
    w = np.ascontiguousarray(w, dtype=np.float64)
    L = w.size - 1
    q = None
    if qids is not None:
        q = np.ascontiguousarray(qids, dtype=np.uint32)
        if q.size != C:
            raise ValueError("need one qid per column")
    st = Stats() if stats else None
    variant = (AGP_VARIANT_INFINITE_TAIL if tail else 0) | (AGP_VARIANT_SPLIT_SIGNS if split_signs else 0)
    if X.dtype == torch.float32:
        fn = lib().agp_propagate_variant if variant else lib().agp_propagate
    elif X.dtype == torch.float64:
        fn = lib().agp_propagate_variant_f64 if variant else lib().agp_propagate_f64
    else:
        raise ValueError("x must be float32 or float64")
    args = [graph.handle, float(a), float(b), w.ctypes.data_as(ct.POINTER(ct.c_double)), L,
            _dptr(X), C, float(eps), ct.c_uint64(int(seed) & 0xFFFFFFFFFFFFFFFF),
            None if q is None else q.ctypes.data_as(ct.POINTER(ct.c_uint32))]
    if variant:
        args.append(variant)
    args += [_dptr(o), _stream_ptr(stream), ct.byref(st) if st is not None else None]
    _check(fn(*args))
    res = o.reshape(-1) if vec else o
    return res, (st.to_dict() if st is not None else None)


def propagate_noalloc(graph: Graph, a: float, b: float, w, x, eps: float, seed: int, *, qids=None, out=None,
                      stream=None):
    """propagate() through agp_propagate_noalloc: binary32, no stats, no
    device allocation inside the call (the library's fixed per-device array
    holds every buffer; at most about 2 million cells n * C).  Pass `out` to
    keep the call itself free of allocations."""
    import torch

    if not x.is_cuda or x.dtype != torch.float32:
        raise ValueError("x must be a float32 device tensor")
    vec = x.dim() == 1
    X = x.reshape(graph.n, -1)
    if not X.is_contiguous():
        raise ValueError("x must be contiguous")
    C = X.shape[1]
    if out is None:
        out = torch.empty_like(X)
    o = out.reshape(graph.n, -1)
    if not o.is_contiguous() or o.dtype != X.dtype or o.shape != X.shape:
        raise ValueError("out must be a contiguous tensor of x's shape and dtype")
    w = np.ascontiguousarray(w, dtype=np.float64)
    q = None
    if qids is not None:
        q = np.ascontiguousarray(qids, dtype=np.uint32)
        if q.size != C:
            raise ValueError("need one qid per column")
    _check(lib().agp_propagate_noalloc(graph.handle, float(a), float(b), w.ctypes.data_as(ct.POINTER(ct.c_double)),
                                       w.size - 1, _dptr(X), C, float(eps),
                                       ct.c_uint64(int(seed) & 0xFFFFFFFFFFFFFFFF),
                                       None if q is None else q.ctypes.data_as(ct.POINTER(ct.c_uint32)), _dptr(o),
                                       _stream_ptr(stream)))
    return o.reshape(-1) if vec else o


TUNING_FIELDS = ("aggregation", "level_blocks", "dense", "tile_columns", "big_row", "big_items",
                 "sparse_shift", "bin_shift", "capture")


class Tuning(ct.Structure):
    _fields_ = [(name, ct.c_int32) for name in TUNING_FIELDS]

    def to_dict(self) -> dict:
        names = {0: "atomic", 1: "binned", 2: "auto"}
        d = {k: int(getattr(self, k)) for k in TUNING_FIELDS}
        d["aggregation"] = names.get(self.aggregation, str(self.aggregation))
        d["dense"] = {0: "never", 1: "always", 2: "auto"}.get(self.dense, str(self.dense))
        return d

    @classmethod
    def from_dict(cls, d: dict) -> "Tuning":
        t = cls()
        agg = {"atomic": 0, "binned": 1, "auto": 2}
        den = {"never": 0, "always": 1, "auto": 2}
        for k in TUNING_FIELDS:
            v = d.get(k, 0)
            if k == "aggregation" and isinstance(v, str):
                v = agg[v]
            if k == "dense" and isinstance(v, str):
                v = den[v]
            setattr(t, k, int(v))
        return t


def _tune_lib():
    L = lib()
    if not getattr(L, "_tune_ready", False):
        vp = ct.c_void_p
        L.agp_autotune.argtypes = [vp, ct.c_double, ct.c_double, ct.POINTER(ct.c_double), ct.c_int32, vp,
                                   ct.c_int32, ct.c_double, ct.c_uint64, ct.POINTER(ct.c_uint32), vp, vp,
                                   ct.POINTER(Tuning)]
        L.agp_get_tuning.argtypes = [vp, ct.c_int32, ct.c_double, ct.c_double, ct.POINTER(Tuning)]
        L.agp_set_tuning.argtypes = [vp, ct.c_int32, ct.c_double, ct.c_double, ct.POINTER(Tuning)]
        L._tune_ready = True
    return L


def autotune(graph: Graph, a: float, b: float, w, x, eps: float, seed: int, *, qids=None, out=None,
             stream=None) -> dict:
    """Time the interchangeable execution choices on this workload (binary32)
    and keep the fastest for later calls with the same C, a, b."""
    import torch

    X = x.reshape(graph.n, -1).contiguous()
    if X.dtype != torch.float32:
        raise ValueError("autotune takes binary32 signals")
    C = X.shape[1]
    o = torch.empty_like(X) if out is None else out.reshape(graph.n, -1)
    w = np.ascontiguousarray(w, dtype=np.float64)
    q = None if qids is None else np.ascontiguousarray(qids, dtype=np.uint32)
    t = Tuning()
    _check(_tune_lib().agp_autotune(graph.handle, float(a), float(b), w.ctypes.data_as(ct.POINTER(ct.c_double)),
                                    w.size - 1, _dptr(X), C, float(eps), ct.c_uint64(int(seed) & 0xFFFFFFFFFFFFFFFF),
                                    None if q is None else q.ctypes.data_as(ct.POINTER(ct.c_uint32)), _dptr(o),
                                    _stream_ptr(stream), ct.byref(t)))
    return t.to_dict()


def get_tuning(graph: Graph, C: int, a: float, b: float) -> dict:
    t = Tuning()
    _check(_tune_lib().agp_get_tuning(graph.handle, int(C), float(a), float(b), ct.byref(t)))
    return t.to_dict()


def set_tuning(graph: Graph, C: int, a: float, b: float, tuning: dict | None) -> None:
    """Pin execution choices (a dict of agp_tuning_t fields; missing ones take
    the defaults) for calls with C columns and exponents a, b; None forgets."""
    t = None if tuning is None else Tuning.from_dict(tuning)
    _check(_tune_lib().agp_set_tuning(graph.handle, int(C), float(a), float(b),
                                      None if t is None else ct.byref(t)))


def sweep(graph: Graph, pi, *, order: bool = True, stream=None):
    """Local clustering sweep (Section 5) of the estimate pi: a float32 CUDA
    tensor of n values, contiguous or a strided column (e.g. out[:, c] of a
    row-major n x C result).  Returns (best_size, best_conductance, order)
    with order an int32 device tensor (None when order=False); the cluster
    is order[:best_size]."""
    import torch

    if not pi.is_cuda or pi.dtype != torch.float32 or pi.dim() != 1 or pi.numel() != graph.n:
        raise ValueError("pi must be a 1-d float32 device tensor of n values")
    ld = pi.stride(0) if graph.n > 1 else 1
    if ld < 1:
        raise ValueError("pi needs a positive stride")
    o = torch.empty(graph.n, dtype=torch.int32, device=pi.device) if order else None
    size = ct.c_int64()
    phi = ct.c_double()
    _check(lib().agp_sweep(graph.handle, _dptr(pi), ld, _stream_ptr(stream), ct.byref(size), ct.byref(phi),
                           None if o is None else _dptr(o)))
    return size.value, phi.value, o


def sweep_batch(graph: Graph, pis, *, stream=None):
    """Sweeps of many estimates at once: pis is a float32 CUDA tensor of
    shape (n, C) whose rows are contiguous (e.g. an agp_propagate result or
    a slice of its columns).  Returns (best_size, best_conductance) as host
    arrays of C entries, each equal to sweep() of that column."""
    import torch

    if not pis.is_cuda or pis.dtype != torch.float32 or pis.dim() != 2 or pis.shape[0] != graph.n:
        raise ValueError("pis must be a 2-d float32 device tensor with n rows")
    C = pis.shape[1]
    if C < 1 or (graph.n > 1 and pis.stride(1) != 1):
        raise ValueError("pis needs at least one column and contiguous rows")
    ld = pis.stride(0) if graph.n > 1 else C
    size = np.zeros(C, dtype=np.int64)
    phi = np.zeros(C, dtype=np.float64)
    _check(lib().agp_sweep_batch(graph.handle, _dptr(pis), max(ld, C), C, _stream_ptr(stream),
                                 size.ctypes.data_as(ct.POINTER(ct.c_int64)),
                                 phi.ctypes.data_as(ct.POINTER(ct.c_double))))
    return size, phi


def device_philox4x32_10(ctr, key) -> np.ndarray:
    """The device Philox4x32-10 blocks of ctr (k x 4) under key (k x 2)."""
    c = np.ascontiguousarray(np.asarray(ctr, dtype=np.uint32).reshape(-1, 4))
    k = np.ascontiguousarray(np.asarray(key, dtype=np.uint32).reshape(-1, 2))
    if c.shape[0] != k.shape[0]:
        raise ValueError("one key per counter block")
    out = np.empty_like(c)
    _check(lib().agp_device_philox4x32_10(c.shape[0], c.ctypes.data, k.ctypes.data, out.ctypes.data))
    return out


def device_splitmix64(values) -> np.ndarray:
    v = np.ascontiguousarray(np.asarray(values, dtype=np.uint64).ravel())
    out = np.empty_like(v)
    _check(lib().agp_device_splitmix64(v.size, v.ctypes.data, out.ctypes.data))
    return out


def _weights(fn, *args, L: int) -> np.ndarray:
    w = np.empty(L + 1, dtype=np.float64)
    _check(fn(*args, L, w.ctypes.data_as(ct.POINTER(ct.c_double))))
    return w


def weights_ppr(alpha: float, L: int) -> np.ndarray:
    return _weights(lib().agp_weights_ppr, float(alpha), L=L)


def weights_hkpr(t: float, L: int) -> np.ndarray:
    return _weights(lib().agp_weights_hkpr, float(t), L=L)


def weights_katz(beta: float, L: int) -> np.ndarray:
    return _weights(lib().agp_weights_katz, float(beta), L=L)


def weights_tp(L: int) -> np.ndarray:
    w = np.empty(L + 1, dtype=np.float64)
    _check(lib().agp_weights_tp(L, w.ctypes.data_as(ct.POINTER(ct.c_double))))
    return w


class Query(ct.Structure):
    _fields_ = [("source", ct.c_int64), ("a", ct.c_double), ("b", ct.c_double), ("L", ct.c_int32),
                ("w", ct.POINTER(ct.c_double)), ("eps", ct.c_double), ("seed", ct.c_uint64),
                ("query_id", ct.c_uint32), ("out", ct.c_void_p), ("x_nnz", ct.c_int64),
                ("x_idx", ct.POINTER(ct.c_int64)), ("x_val", ct.POINTER(ct.c_float))]


class ServerConfig(ct.Structure):
    _fields_ = [("max_slots", ct.c_int32), ("queue_capacity", ct.c_int32), ("work_budget", ct.c_double),
                ("memory_bytes", ct.c_int64)]


class Result(ct.Structure):
    _fields_ = [("status", ct.c_int32), ("levels", ct.c_int32), ("frontier", ct.c_uint64),
                ("pushes", ct.c_uint64), ("candidates", ct.c_uint64), ("table_entries", ct.c_uint64),
                ("restarts", ct.c_int32), ("submit_ms", ct.c_double),
                ("start_ms", ct.c_double), ("end_ms", ct.c_double)]

    def to_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


def _server_lib():
    L = lib()
    if not getattr(L, "_server_ready", False):
        vp = ct.c_void_p
        L.agp_server_create.argtypes = [vp, ct.POINTER(ServerConfig), ct.POINTER(vp)]
        L.agp_submit.argtypes = [vp, ct.POINTER(Query), ct.POINTER(ct.c_uint64)]
        L.agp_poll.argtypes = [vp, ct.c_uint64, ct.POINTER(Result)]
        L.agp_server_destroy.argtypes = [vp]
        L._server_ready = True
    return L


class Server:
    """Continuous-batching server of single-source queries on one graph."""

    def __init__(self, graph: Graph, max_slots: int = 64, queue_capacity: int = 4096,
                 work_budget: float = 0.0, memory_bytes: int = 0):
        """memory_bytes: device memory of the running queries' residue tables
        (0: a quarter of the free device memory)."""
        L = _server_lib()
        self.graph = graph  # keeps the graph alive
        cfg = ServerConfig(max_slots, queue_capacity, work_budget, int(memory_bytes))
        h = ct.c_void_p()
        _check(L.agp_server_create(graph.handle, ct.byref(cfg), ct.byref(h)))
        self._h = h

    def submit(self, source: int, a: float, b: float, w, eps: float, seed: int, query_id: int, out,
               x=None) -> int:
        """Queue a query with signal e_source, or with the sparse signal
        x = (ids, values) when x is given (source is then ignored)."""
        w = np.ascontiguousarray(w, dtype=np.float64)
        q = Query(int(source), float(a), float(b), w.size - 1, w.ctypes.data_as(ct.POINTER(ct.c_double)),
                  float(eps), ct.c_uint64(int(seed) & 0xFFFFFFFFFFFFFFFF), int(query_id), _dptr(out))
        if x is not None:
            idx = np.ascontiguousarray(x[0], dtype=np.int64)
            val = np.ascontiguousarray(x[1], dtype=np.float32)
            if idx.size != val.size:
                raise ValueError("x needs as many ids as values")
            q.x_nnz = idx.size
            q.x_idx = idx.ctypes.data_as(ct.POINTER(ct.c_int64))
            q.x_val = val.ctypes.data_as(ct.POINTER(ct.c_float))
        t = ct.c_uint64()
        _check(_server_lib().agp_submit(self._h, ct.byref(q), ct.byref(t)))
        return t.value

    def poll(self, ticket: int):
        """Result dict when finished, None while pending (raises on unknown tickets)."""
        r = Result()
        rc = _server_lib().agp_poll(self._h, ticket, ct.byref(r))
        if rc == AGP_PENDING:
            return None
        _check(rc)
        return r.to_dict()

    def close(self) -> None:
        if getattr(self, "_h", None) is not None:
            _server_lib().agp_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
