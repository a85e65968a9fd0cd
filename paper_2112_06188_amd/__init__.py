"""MI355X BDL-tree: Python binding of the C ABI in include/bdl.h.

The binding only marshals arguments: torch supplies device memory and the
stream, and every step of Insert_L, Erase_L and kNN_L runs in the HIP
kernels of libbdl.so.  Importing works without a GPU (so that the library's
exports can be inspected); creating a tree needs the built library and a
GPU, and fails loudly otherwise.
"""
from __future__ import annotations

import ctypes
import os
from typing import Dict, Optional, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbdl.so")

BDL_OK = 0
BDL_EINVAL = -1
BDL_ENOMEM = -2
BDL_EHIP = -3
MAX_DIM = 16
MAX_K = 64
INVALID_ID = 0xFFFFFFFF
FLAG_CHECK_INPUTS = 1

# Every symbol include/bdl.h and include/bdl_server.h declare.
EXPORTS = [
    "bdl_create", "bdl_insert", "bdl_erase", "bdl_knn", "bdl_clear", "bdl_sync", "bdl_destroy",
    "bdl_size", "bdl_level_info", "bdl_counters", "bdl_debug_export_level",
    "bdl_debug_export_buffer", "bdl_last_error", "bdl_profile", "bdl_level_sizes",
    "bdl_set_param", "bdl_knn_batch", "bdl_set_knn_shapes",
    "bdl_server_create", "bdl_server_submit", "bdl_server_wait", "bdl_server_poll",
    "bdl_server_drain", "bdl_server_destroy", "bdl_knn_noalloc", "bdl_host_waits",
    "bdl_knn_graph",
]
REQ_KNN, REQ_INSERT, REQ_ERASE = 0, 1, 2
SERVE_FIFO, SERVE_BATCHED = 0, 1
FLAG_PROFILE = 2
FLAG_OBJECT_MEDIAN = 4  # split heuristic: object median instead of spatial (Section V-C)
FLAG_REBUILD_ALL = 8    # baseline B1 of Section III-B instead of the BDL-tree
FLAG_NO_REBUILD = 16    # baseline B2 of Section III-B instead of the BDL-tree
STRUCTURES = {"bdl": 0, "rebuild_all": FLAG_REBUILD_ALL, "no_rebuild": FLAG_NO_REBUILD}
PARAM_KNN_KERNEL = 1
PARAM_SORT_MIN = 2
PARAM_KNN_BLOCK = 3
PARAM_USE_GRAPHS = 4
PARAM_PERSISTENT = 5
PARAM_QUERY_MAX = 6
PARAM_QUERY_STACK = 7
PARAM_ERASE_ROUTE = 8
PARAM_GRAPH_START = 9
MAX_SHAPES = 256
KNN_LANE = 0
KNN_WAVE = 1
KNN_AUTO = 2
KNN_QUERY = 3
PHASES = ["gather", "passes", "finish", "layout", "erase", "order", "traverse", "other"]


class Profile(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double * 8), ("calls", ctypes.c_int64 * 8),
                ("knn_nodes", ctypes.c_int64), ("knn_leaves", ctypes.c_int64),
                ("knn_points", ctypes.c_int64)]

NODE_DTYPE = np.dtype([
    ("lo", np.float32, (MAX_DIM,)),
    ("hi", np.float32, (MAX_DIM,)),
    ("split", np.float32),
    ("dim", np.int32),
    ("left", np.int32),
    ("right", np.int32),
    ("parent", np.int32),
    ("begin", np.int32),
    ("count", np.int32),
    ("depth", np.int32),
    ("pad_", np.int32),
    ("path", np.uint64),
], align=True)


class KnnRequest(ctypes.Structure):
    _fields_ = [("q", ctypes.c_void_p), ("nq", ctypes.c_int64), ("k", ctypes.c_int32),
                ("pad_", ctypes.c_int32), ("out_ids", ctypes.c_void_p),
                ("out_d2", ctypes.c_void_p)]


class KnnShape(ctypes.Structure):
    """One row of the k-NN launch-shape table (bdl_knn_shape)."""
    _fields_ = [("k_lo", ctypes.c_int32), ("k_hi", ctypes.c_int32),
                ("nq_lo", ctypes.c_int64), ("nq_hi", ctypes.c_int64),
                ("kernel", ctypes.c_int32), ("block", ctypes.c_int32),
                ("persistent", ctypes.c_int32), ("sort", ctypes.c_int32)]


class ServerConfig(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("max_inflight", ctypes.c_int32),
                ("max_batch_requests", ctypes.c_int32), ("max_launches", ctypes.c_int32),
                ("max_batch_queries", ctypes.c_int64), ("mem_budget", ctypes.c_uint64)]


class Request(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("k", ctypes.c_int32), ("n", ctypes.c_int64),
                ("pts", ctypes.c_void_p), ("ids", ctypes.c_void_p),
                ("out_ids", ctypes.c_void_p), ("out_d2", ctypes.c_void_p)]


class Completion(ctypes.Structure):
    _fields_ = [("ticket", ctypes.c_uint64), ("admit_seq", ctypes.c_uint64),
                ("kind", ctypes.c_int32), ("status", ctypes.c_int32),
                ("n_erased", ctypes.c_int64), ("launch", ctypes.c_int64),
                ("t_submit_ms", ctypes.c_double), ("t_admit_ms", ctypes.c_double),
                ("t_start_ms", ctypes.c_double), ("t_done_ms", ctypes.c_double)]


class BdlError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"bdl error {code}: {msg}")
        self.code = code


class Config(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int32),
        ("leaf_size", ctypes.c_int32),
        ("buffer_size", ctypes.c_int32),
        ("id_capacity", ctypes.c_uint32),
        ("mem_budget", ctypes.c_uint64),
        ("flags", ctypes.c_uint32),
    ]


_lib = None


def load_library(path: Optional[str] = None):
    """Load libbdl.so (or the library BDL_LIBRARY names) and declare its
    signatures (no GPU needed)."""
    global _lib
    if _lib is not None:
        return _lib
    path = path or os.environ.get("BDL_LIBRARY") or LIB_PATH
    if not os.path.exists(path):
        raise FileNotFoundError(
            f"{path} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'`")
    lib = ctypes.CDLL(path)
    vp, i64, i32, u32p, f32p = (ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
                               ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(ctypes.c_float))
    i64p = ctypes.POINTER(ctypes.c_int64)
    lib.bdl_create.argtypes = [ctypes.POINTER(Config), vp, ctypes.POINTER(vp)]
    lib.bdl_insert.argtypes = [vp, vp, vp, i64]
    lib.bdl_erase.argtypes = [vp, vp, vp, i64, i64p]
    lib.bdl_knn.argtypes = [vp, vp, i64, i32, vp, vp]
    lib.bdl_knn_noalloc.argtypes = [vp, vp, i64, i32, vp, vp]
    lib.bdl_knn_graph.argtypes = [vp, i32, vp, vp]
    lib.bdl_sync.argtypes = [vp]
    lib.bdl_clear.argtypes = [vp]
    lib.bdl_set_param.argtypes = [vp, i32, i64]
    lib.bdl_knn_batch.argtypes = [vp, ctypes.POINTER(KnnRequest), i32]
    lib.bdl_set_knn_shapes.argtypes = [vp, ctypes.POINTER(KnnShape), i32]
    lib.bdl_profile.argtypes = [vp, ctypes.POINTER(Profile), ctypes.c_int]
    lib.bdl_destroy.argtypes = [vp]
    lib.bdl_destroy.restype = None
    lib.bdl_size.argtypes = [vp]
    lib.bdl_size.restype = i64
    lib.bdl_level_info.argtypes = [vp, ctypes.POINTER(i32), i64p, i64p, i64p,
                                   ctypes.POINTER(ctypes.c_uint64)]
    lib.bdl_counters.argtypes = [vp, i64p, i64p]
    lib.bdl_host_waits.argtypes = [vp, i64p]
    lib.bdl_host_waits.restype = ctypes.c_int
    lib.bdl_level_sizes.argtypes = [vp, ctypes.POINTER(i32), i64p, i64p, i64p]
    lib.bdl_debug_export_level.argtypes = [vp, i32, u32p, f32p, vp, i64p, i64p]
    lib.bdl_debug_export_buffer.argtypes = [vp, u32p, f32p, i64p]
    lib.bdl_last_error.restype = ctypes.c_char_p
    lib.bdl_server_create.argtypes = [vp, ctypes.POINTER(ServerConfig), ctypes.POINTER(vp)]
    lib.bdl_server_submit.argtypes = [vp, ctypes.POINTER(Request),
                                      ctypes.POINTER(ctypes.c_uint64)]
    lib.bdl_server_wait.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(Completion)]
    lib.bdl_server_poll.argtypes = [vp, ctypes.POINTER(Completion), i32, ctypes.POINTER(i32)]
    lib.bdl_server_drain.argtypes = [vp]
    lib.bdl_server_destroy.argtypes = [vp]
    lib.bdl_server_destroy.restype = None
    for name in ("bdl_create", "bdl_insert", "bdl_erase", "bdl_knn", "bdl_knn_noalloc",
                 "bdl_clear", "bdl_sync",
                 "bdl_profile", "bdl_level_sizes", "bdl_set_param", "bdl_knn_batch",
                 "bdl_set_knn_shapes", "bdl_server_create", "bdl_server_submit",
                 "bdl_server_wait", "bdl_server_poll", "bdl_server_drain",
                 "bdl_level_info", "bdl_counters", "bdl_debug_export_level",
                 "bdl_debug_export_buffer"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _check(rc: int) -> None:
    if rc != 0:
        msg = _lib.bdl_last_error().decode(errors="replace")
        raise BdlError(rc, msg)


def _torch():
    import torch
    return torch


class Tree:
    """A BDL-tree resident in HBM of one GPU.

    split selects the build heuristic of Section V-C: "spatial" (midpoint of
    a node's extent, the default) or "object" (median of its coordinates).
    structure selects the BDL-tree ("bdl", the default) or one of the
    baselines of Section III-B: "rebuild_all" (B1) or "no_rebuild" (B2).
    Points and queries are CUDA (HIP) float32 tensors of shape [n, dim];
    ids are int32 or uint32 tensors holding the uint32 ids bit for bit.
    All work is ordered on the stream that is current at construction.
    """

    def __init__(self, dim: int, leaf_size: int = 16, buffer_size: int = 1024,
                 id_capacity: int = 1 << 24, mem_budget: int = 0, check_inputs: bool = False,
                 profile: bool = False, device: Optional[int] = None, stream=None,
                 split: str = "spatial", structure: str = "bdl"):
        torch = _torch()
        lib = load_library()
        if not torch.cuda.is_available():
            raise RuntimeError("a GPU is required: the BDL-tree runs only in HIP kernels")
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        self.dim = int(dim)
        self.leaf_size = int(leaf_size)
        self.buffer_size = int(buffer_size)
        self.id_capacity = int(id_capacity)
        with torch.cuda.device(self.device):
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
            if split not in ("spatial", "object"):
                raise ValueError(f"split must be 'spatial' or 'object', not {split!r}")
            if structure not in STRUCTURES:
                raise ValueError(f"structure must be one of {sorted(STRUCTURES)}, not {structure!r}")
            flags = (FLAG_CHECK_INPUTS if check_inputs else 0) | (FLAG_PROFILE if profile else 0) \
                | (FLAG_OBJECT_MEDIAN if split == "object" else 0) | STRUCTURES[structure]
            cfg = Config(self.dim, self.leaf_size, self.buffer_size, self.id_capacity,
                         int(mem_budget), flags)
            h = ctypes.c_void_p()
            _check(lib.bdl_create(ctypes.byref(cfg), ctypes.c_void_p(self.stream.cuda_stream),
                                  ctypes.byref(h)))
        self._h = h
        self._lib = lib

    # -- lifetime --------------------------------------------------------
    def close(self) -> None:
        if getattr(self, "_h", None):
            self._lib.bdl_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- marshalling -----------------------------------------------------
    def _pts(self, x, name: str):
        torch = _torch()
        if not isinstance(x, torch.Tensor):
            x = torch.as_tensor(np.ascontiguousarray(x, dtype=np.float32))
        if x.dtype != torch.float32:
            raise TypeError(f"{name} must be float32")
        if x.dim() != 2 or x.shape[1] != self.dim:
            raise ValueError(f"{name} must have shape [n, {self.dim}]")
        return x.to(self.device).contiguous()

    def _ids(self, x, n: int):
        torch = _torch()
        if not isinstance(x, torch.Tensor):
            x = torch.from_numpy(np.ascontiguousarray(x, dtype=np.uint32).view(np.int32))
        if x.dtype not in (torch.int32, getattr(torch, "uint32", torch.int32)):
            raise TypeError("ids must be int32 or uint32")
        x = x.reshape(-1)
        if x.shape[0] != n:
            raise ValueError("ids and points differ in length")
        return x.to(self.device).contiguous()

    # -- operations ------------------------------------------------------
    def insert(self, pts, ids) -> None:
        """Insert_L (Alg. 3)."""
        p = self._pts(pts, "pts")
        i = self._ids(ids, p.shape[0])
        with _torch().cuda.device(self.device):
            _check(self._lib.bdl_insert(self._h, ctypes.c_void_p(p.data_ptr()),
                                        ctypes.c_void_p(i.data_ptr()), p.shape[0]))
            self._keep_on_stream(p, i)

    def erase(self, pts, ids) -> int:
        """Erase_L (Alg. 4); returns the number of points erased."""
        p = self._pts(pts, "pts")
        i = self._ids(ids, p.shape[0])
        out = ctypes.c_int64()
        with _torch().cuda.device(self.device):
            _check(self._lib.bdl_erase(self._h, ctypes.c_void_p(p.data_ptr()),
                                       ctypes.c_void_p(i.data_ptr()), p.shape[0],
                                       ctypes.byref(out)))
        return int(out.value)

    def _out(self, x, nq: int, k: int, dtype, name: str):
        """A caller-supplied output must be a contiguous [nq, k] tensor of
        the right dtype on this tree's device; a new one is allocated when
        x is None."""
        torch = _torch()
        if x is None:
            return torch.empty((nq, k), dtype=dtype, device=self.device)
        if not isinstance(x, torch.Tensor) or x.dtype != dtype or tuple(x.shape) != (nq, k) \
                or x.device != self.device or not x.is_contiguous():
            raise ValueError(f"{name} must be a contiguous {dtype} tensor of shape "
                             f"[{nq}, {k}] on {self.device}")
        return x

    def _keep_on_stream(self, *tensors) -> None:
        """The library reads and writes these on the tree's stream after the
        call returns: keep the caching allocator from reusing them before
        that stream passes this point."""
        torch = _torch()
        if self.stream != torch.cuda.current_stream(self.device):
            for x in tensors:
                x.record_stream(self.stream)

    def knn(self, q, k: int, out_ids=None, out_d2=None):
        """kNN_L (Alg. 5): (ids int32 [nq, k], squared distances float32 [nq, k])."""
        return self._knn(self._lib.bdl_knn, q, k, out_ids, out_d2)

    def knn_noalloc(self, q, k: int, out_ids=None, out_d2=None):
        """kNN_L through bdl_knn_noalloc (no device allocation by the library;
        at most 1048576 queries per call)."""
        return self._knn(self._lib.bdl_knn_noalloc, q, k, out_ids, out_d2)

    def knn_graph(self, k: int, out_ids=None, out_d2=None):
        """The k-NN graph of the live points (bdl_knn_graph): row `id` of
        (ids int32 [id_capacity, k], squared distances float32 [id_capacity,
        k]) holds the row kNN_L returns for live point `id` as a query.
        Rows of ids that are not live are left as they were: when the
        outputs are allocated here, ids -1 and distances +inf."""
        torch = _torch()
        n = self.id_capacity
        if out_ids is None:
            out_ids = torch.full((n, k), -1, dtype=torch.int32, device=self.device)
        if out_d2 is None:
            out_d2 = torch.full((n, k), float("inf"), dtype=torch.float32, device=self.device)
        out_ids = self._out(out_ids, n, k, torch.int32, "out_ids")
        out_d2 = self._out(out_d2, n, k, torch.float32, "out_d2")
        with torch.cuda.device(self.device):
            _check(self._lib.bdl_knn_graph(self._h, int(k), ctypes.c_void_p(out_ids.data_ptr()),
                                           ctypes.c_void_p(out_d2.data_ptr())))
            self._keep_on_stream(out_ids, out_d2)
        return out_ids, out_d2

    def _knn(self, fn, q, k: int, out_ids, out_d2):
        torch = _torch()
        qq = self._pts(q, "q")
        nq = qq.shape[0]
        out_ids = self._out(out_ids, nq, k, torch.int32, "out_ids")
        out_d2 = self._out(out_d2, nq, k, torch.float32, "out_d2")
        with torch.cuda.device(self.device):
            _check(fn(self._h, ctypes.c_void_p(qq.data_ptr()), nq, int(k),
                      ctypes.c_void_p(out_ids.data_ptr()), ctypes.c_void_p(out_d2.data_ptr())))
            self._keep_on_stream(qq, out_ids, out_d2)
        return out_ids, out_d2

    def knn_batch(self, requests, outputs=None):
        """Batched kNN_L: requests is a list of (queries, k); returns a list of
        (ids, d2) pairs, the same as knn() on each request in turn."""
        torch = _torch()
        reqs = (KnnRequest * max(1, len(requests)))()
        keep = []
        outs = []
        for i, (q, k) in enumerate(requests):
            qq = self._pts(q, "q")
            nq = qq.shape[0]
            oi, od = outputs[i] if outputs is not None else (None, None)
            oi = self._out(oi, nq, k, torch.int32, f"outputs[{i}] ids")
            od = self._out(od, nq, k, torch.float32, f"outputs[{i}] d2")
            keep += [qq, oi, od]
            outs.append((oi, od))
            reqs[i] = KnnRequest(qq.data_ptr(), nq, int(k), 0, oi.data_ptr(), od.data_ptr())
        with torch.cuda.device(self.device):
            _check(self._lib.bdl_knn_batch(self._h, reqs, len(requests)))
            self._keep_on_stream(*keep)
        return outs

    def sync(self) -> None:
        _check(self._lib.bdl_sync(self._h))

    def profile(self, reset: bool = False) -> Dict[str, Dict[str, float]]:
        """Per-phase device milliseconds and call counts (BDL_FLAG_PROFILE)."""
        p = Profile()
        _check(self._lib.bdl_profile(self._h, ctypes.byref(p), 1 if reset else 0))
        out = {name: {"ms": p.ms[i], "calls": p.calls[i]} for i, name in enumerate(PHASES)}
        out["knn_work"] = {"nodes": p.knn_nodes, "leaves": p.knn_leaves, "points": p.knn_points}
        return out

    def set_param(self, param: int, value: int) -> None:
        """Tuning knobs (PARAM_*); they change speed, never results."""
        _check(self._lib.bdl_set_param(self._h, int(param), int(value)))

    def set_knn_shapes(self, rows) -> None:
        """Install a k-NN launch-shape table: rows of dicts (or tuples in
        KnnShape field order) with k_lo, k_hi, nq_lo, nq_hi, kernel, block,
        persistent, sort.  An empty list removes the table."""
        rows = list(rows)
        arr = (KnnShape * max(1, len(rows)))()
        names = [f for f, _ in KnnShape._fields_]
        for i, r in enumerate(rows):
            vals = [r[n] for n in names] if isinstance(r, dict) else list(r)
            for n, v in zip(names, vals):
                setattr(arr[i], n, int(v))
        _check(self._lib.bdl_set_knn_shapes(self._h, arr, len(rows)))
        self._shapes = [dict(zip(names, (getattr(arr[i], n) for n in names)))
                        for i in range(len(rows))]

    def clear(self) -> None:
        """Remove every point; device memory is kept for reuse."""
        _check(self._lib.bdl_clear(self._h))

    def size(self) -> int:
        return int(self._lib.bdl_size(self._h))

    def level_info(self) -> Dict:
        nlev = ctypes.c_int32()
        live = np.zeros(64, np.int64)
        cap = np.zeros(64, np.int64)
        buf = ctypes.c_int64()
        F = ctypes.c_uint64()
        p64 = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
        _check(self._lib.bdl_level_info(self._h, ctypes.byref(nlev), p64(live), p64(cap),
                                        ctypes.byref(buf), ctypes.byref(F)))
        n = nlev.value
        return {"nlev": n, "live": live[:n].copy(), "cap": cap[:n].copy(),
                "buf_live": buf.value, "F": F.value}

    def level_sizes(self) -> Dict:
        nlev = ctypes.c_int32()
        slots = np.zeros(64, np.int64)
        nodes = np.zeros(64, np.int64)
        bnodes = ctypes.c_int64()
        p64 = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
        _check(self._lib.bdl_level_sizes(self._h, ctypes.byref(nlev), p64(slots), p64(nodes),
                                         ctypes.byref(bnodes)))
        n = nlev.value
        return {"slots": slots[:n].copy(), "nodes": nodes[:n].copy(), "buf_nodes": bnodes.value}

    def host_waits(self) -> int:
        """Times the library has blocked the host on the tree's stream."""
        w = ctypes.c_int64()
        _check(self._lib.bdl_host_waits(self._h, ctypes.byref(w)))
        return int(w.value)

    def counters(self) -> Dict:
        rb = ctypes.c_int64()
        ri = ctypes.c_int64()
        _check(self._lib.bdl_counters(self._h, ctypes.byref(rb), ctypes.byref(ri)))
        return {"rebuilt": rb.value, "reinserted": ri.value}

    def export_level(self, level: int) -> Optional[Tuple[np.ndarray, np.ndarray, np.ndarray]]:
        """(ids uint32 [n], pts float32 [n, d], nodes NODE_DTYPE [m]) of static tree
        `level` (-1: the buffer's tree), or None if that tree is empty."""
        ns = ctypes.c_int64()
        nn = ctypes.c_int64()
        rc = self._lib.bdl_debug_export_level(self._h, level, None, None, None,
                                              ctypes.byref(ns), ctypes.byref(nn))
        if rc != 0 or ns.value == 0:
            return None
        ids = np.empty(ns.value, np.uint32)
        pts = np.empty((ns.value, self.dim), np.float32)
        nodes = np.empty(nn.value, NODE_DTYPE)
        _check(self._lib.bdl_debug_export_level(
            self._h, level, ids.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
            pts.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
            nodes.ctypes.data_as(ctypes.c_void_p), ctypes.byref(ns), ctypes.byref(nn)))
        return ids, pts, nodes

    def export_buffer(self) -> Tuple[np.ndarray, np.ndarray]:
        n = ctypes.c_int64()
        _check(self._lib.bdl_debug_export_buffer(self._h, None, None, ctypes.byref(n)))
        ids = np.empty(n.value, np.uint32)
        pts = np.empty((n.value, self.dim), np.float32)
        if n.value:
            _check(self._lib.bdl_debug_export_buffer(
                self._h, ids.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
                pts.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), ctypes.byref(n)))
        return ids, pts


def build(verbose: bool = False) -> str:
    from .build_lib import build as _b
    return _b(verbose=verbose)


def _completion_dict(c: "Completion") -> Dict:
    return {f: getattr(c, f) for f, _ in Completion._fields_}


class Server:
    """Served form (include/bdl_server.h): a native request loop over `tree`.

    Requests carry host (numpy) arrays; submit_* return a ticket, wait()
    returns the completion (and, for k-NN, the (ids, d2) arrays).  While the
    server exists only its loop uses the tree.
    """

    def __init__(self, tree: "Tree", mode: int = SERVE_BATCHED, max_inflight: int = 4096,
                 max_batch_requests: int = 4096, max_batch_queries: int = 1 << 22,
                 max_launches: int = 2, mem_budget: int = 0):
        self._lib = load_library()
        self.tree = tree
        self.dim = tree.dim
        cfg = ServerConfig(int(mode), int(max_inflight), int(max_batch_requests),
                           int(max_launches), int(max_batch_queries), int(mem_budget))
        h = ctypes.c_void_p()
        _check(self._lib.bdl_server_create(tree._h, ctypes.byref(cfg), ctypes.byref(h)))
        self._h = h
        self._held = {}

    def _submit(self, kind, pts, ids=None, k=0):
        pts = np.ascontiguousarray(pts, dtype=np.float32).reshape(-1, self.dim)
        n = pts.shape[0]
        r = Request(kind, int(k), n, pts.ctypes.data, None, None, None)
        keep = [pts]
        if kind == REQ_KNN:
            oi = np.empty((n, k), np.uint32)
            od = np.empty((n, k), np.float32)
            r.out_ids, r.out_d2 = oi.ctypes.data, od.ctypes.data
            keep += [oi, od]
        else:
            ids = np.ascontiguousarray(ids, dtype=np.uint32).reshape(-1)
            if ids.shape[0] != n:
                raise ValueError("ids and points differ in length")
            r.ids = ids.ctypes.data
            keep.append(ids)
        t = ctypes.c_uint64()
        _check(self._lib.bdl_server_submit(self._h, ctypes.byref(r), ctypes.byref(t)))
        self._held[t.value] = keep
        return t.value

    def submit_knn(self, q, k: int) -> int:
        return self._submit(REQ_KNN, q, k=k)

    def submit_insert(self, pts, ids) -> int:
        return self._submit(REQ_INSERT, pts, ids)

    def submit_erase(self, pts, ids) -> int:
        return self._submit(REQ_ERASE, pts, ids)

    def _finish(self, c: "Completion") -> Dict:
        out = _completion_dict(c)
        keep = self._held.pop(c.ticket, None)
        if c.kind == REQ_KNN and keep is not None:
            out["ids"], out["d2"] = keep[1], keep[2]
        return out

    def wait(self, ticket: int) -> Dict:
        c = Completion()
        _check(self._lib.bdl_server_wait(self._h, int(ticket), ctypes.byref(c)))
        return self._finish(c)

    def poll(self, max_n: int = 1024):
        arr = (Completion * max_n)()
        n = ctypes.c_int32()
        _check(self._lib.bdl_server_poll(self._h, arr, max_n, ctypes.byref(n)))
        return [self._finish(arr[i]) for i in range(n.value)]

    def drain(self) -> None:
        _check(self._lib.bdl_server_drain(self._h))

    def close(self) -> None:
        if getattr(self, "_h", None):
            self._lib.bdl_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
