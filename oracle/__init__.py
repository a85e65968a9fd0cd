"""ctypes wrapper over the serial CPU oracle (``bdl_oracle.c``).

TEST INFRASTRUCTURE ONLY: the oracle is the reference the GPU library is
checked against.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg import this module; the GPU library never does.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading
from typing import Dict, Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bdl_oracle.c")
_LIB = os.path.join(_HERE, "libbdl_oracle.so")
_lock = threading.Lock()
_lib = None

TOMB = 0xFFFFFFFF
MAXD = 16
SPLIT_RULES = {"spatial": 0, "object": 1}  # the two heuristics of Section V-C
# the BDL-tree and the two baselines of Section III-B (B1, B2)
MODES = {"bdl": 0, "rebuild_all": 1, "no_rebuild": 2}
MAX_DEPTH = 63

NODE_DTYPE = np.dtype([
    ("lo", np.float32, (MAXD,)),
    ("hi", np.float32, (MAXD,)),
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

CFLAGS = ["-O3", "-std=c99", "-Wall", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
          "-fPIC", "-shared"]


def build(force: bool = True) -> str:
    """Compile the oracle into a shared library next to its source."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + f".tmp{os.getpid()}"
    subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        c_f = ctypes.POINTER(ctypes.c_float)
        c_u = ctypes.POINTER(ctypes.c_uint32)
        c_i64 = ctypes.POINTER(ctypes.c_int64)
        c_v = ctypes.c_void_p
        lib.orc_create.restype = c_v
        lib.orc_create.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int]
        lib.orc_destroy.argtypes = [c_v]
        lib.orc_insert.argtypes = [c_v, c_f, c_u, ctypes.c_int64]
        lib.orc_erase.restype = ctypes.c_int64
        lib.orc_erase.argtypes = [c_v, c_f, c_u, ctypes.c_int64]
        lib.orc_knn.argtypes = [c_v, c_f, ctypes.c_int64, ctypes.c_int, c_u, c_f, c_v]
        lib.orc_knn_parallel.restype = ctypes.c_int
        lib.orc_knn_parallel.argtypes = [c_v, c_f, ctypes.c_int64, ctypes.c_int, c_u, c_f, c_v]
        lib.orc_size.restype = ctypes.c_int64
        lib.orc_size.argtypes = [c_v]
        lib.orc_level_info.argtypes = [c_v, ctypes.POINTER(ctypes.c_int32), c_i64, c_i64,
                                       c_i64, c_i64, ctypes.POINTER(ctypes.c_uint64),
                                       c_i64, c_i64]
        lib.orc_export_level.argtypes = [c_v, ctypes.c_int32, c_u, c_f, c_v, c_i64, c_i64]
        lib.orc_export_buffer_pool.argtypes = [c_v, c_u, c_f, c_i64]
        lib.orc_set_mode.restype = ctypes.c_int
        lib.orc_set_mode.argtypes = [c_v, ctypes.c_int]
        lib.orc_set_split_rule.restype = ctypes.c_int
        lib.orc_set_split_rule.argtypes = [c_v, ctypes.c_int]
        lib.orc_tree_build_rule.restype = ctypes.c_int64
        lib.orc_tree_build_rule.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, c_f, c_u,
                                            ctypes.c_int64, c_v, ctypes.POINTER(ctypes.c_int32)]
        lib.orc_tree_build.restype = ctypes.c_int64
        lib.orc_tree_build.argtypes = [ctypes.c_int, ctypes.c_int, c_f, c_u, ctypes.c_int64,
                                       c_v, ctypes.POINTER(ctypes.c_int32)]
        lib.orc_bruteforce_knn.argtypes = [ctypes.c_int, c_f, c_u, ctypes.c_int64, c_f,
                                           ctypes.c_int64, ctypes.c_int, c_u, c_f]
        lib.orc_dist2.restype = ctypes.c_float
        lib.orc_dist2.argtypes = [ctypes.c_int, c_f, c_f]
        lib.orc_sizeof_node.restype = ctypes.c_int32
        if lib.orc_sizeof_node() != NODE_DTYPE.itemsize:
            raise RuntimeError("oracle node struct does not match NODE_DTYPE")
        _lib = lib
        return lib


def _fp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


def _up(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))


def _pts(a, d: int) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.float32)
    return a.reshape(-1, d)


def _ids(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.uint32).reshape(-1)


class Counters(ctypes.Structure):
    _fields_ = [("node_visits", ctypes.c_int64), ("dist_evals", ctypes.c_int64)]


class OracleBDL:
    """The log structure of static kd-trees, serial."""

    def __init__(self, dim: int, leaf_size: int = 16, buffer_size: int = 1024,
                 split: str = "spatial", mode: str = "bdl"):
        self._lib = _load()
        self.dim = dim
        self.leaf_size = leaf_size
        self.buffer_size = buffer_size
        self._h = self._lib.orc_create(dim, leaf_size, buffer_size)
        if not self._h:
            raise ValueError("invalid oracle configuration")
        if split not in SPLIT_RULES or self._lib.orc_set_split_rule(self._h, SPLIT_RULES[split]):
            raise ValueError(f"unknown split rule {split!r}")
        if mode not in MODES or self._lib.orc_set_mode(self._h, MODES[mode]):
            raise ValueError(f"unknown structure {mode!r}")

    def close(self) -> None:
        if self._h:
            self._lib.orc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def insert(self, pts, ids) -> None:
        p = _pts(pts, self.dim)
        i = _ids(ids)
        assert p.shape[0] == i.shape[0]
        self._lib.orc_insert(self._h, _fp(p), _up(i), p.shape[0])

    def erase(self, pts, ids) -> int:
        p = _pts(pts, self.dim)
        i = _ids(ids)
        assert p.shape[0] == i.shape[0]
        return int(self._lib.orc_erase(self._h, _fp(p), _up(i), p.shape[0]))

    def knn(self, q, k: int, counters: bool = False):
        qq = _pts(q, self.dim)
        nq = qq.shape[0]
        ids = np.empty((nq, k), dtype=np.uint32)
        d2 = np.empty((nq, k), dtype=np.float32)
        c = Counters()
        self._lib.orc_knn(self._h, _fp(qq), nq, k, _up(ids), _fp(d2), ctypes.byref(c))
        if counters:
            return ids, d2, {"node_visits": c.node_visits, "dist_evals": c.dist_evals}
        return ids, d2

    def knn_parallel(self, q, k: int):
        """The same rows as knn(), with the queries spread over host threads
        (OpenMP; OMP_NUM_THREADS sets the count).  Returns (ids, d2,
        threads used, counters)."""
        qq = _pts(q, self.dim)
        nq = qq.shape[0]
        ids = np.empty((nq, k), dtype=np.uint32)
        d2 = np.empty((nq, k), dtype=np.float32)
        c = Counters()
        used = self._lib.orc_knn_parallel(self._h, _fp(qq), nq, k, _up(ids), _fp(d2),
                                          ctypes.byref(c))
        return ids, d2, int(used), {"node_visits": c.node_visits, "dist_evals": c.dist_evals}

    def size(self) -> int:
        return int(self._lib.orc_size(self._h))

    def level_info(self) -> Dict:
        nlev = ctypes.c_int32()
        live = np.zeros(64, np.int64)
        cap = np.zeros(64, np.int64)
        slots = np.zeros(64, np.int64)
        buf = ctypes.c_int64()
        F = ctypes.c_uint64()
        rb = ctypes.c_int64()
        ri = ctypes.c_int64()
        p64 = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
        self._lib.orc_level_info(self._h, ctypes.byref(nlev), p64(live), p64(cap), p64(slots),
                                 ctypes.byref(buf), ctypes.byref(F), ctypes.byref(rb),
                                 ctypes.byref(ri))
        n = nlev.value
        return {"nlev": n, "live": live[:n].copy(), "cap": cap[:n].copy(),
                "slots": slots[:n].copy(), "buf_live": buf.value, "F": F.value,
                "rebuilt": rb.value, "reinserted": ri.value}

    def export_level(self, level: int) -> Optional[Tuple[np.ndarray, np.ndarray, np.ndarray]]:
        ns = ctypes.c_int64()
        nn = ctypes.c_int64()
        rc = self._lib.orc_export_level(self._h, level, None, None, None,
                                        ctypes.byref(ns), ctypes.byref(nn))
        if rc != 0:
            return None
        ids = np.empty(ns.value, np.uint32)
        pts = np.empty((ns.value, self.dim), np.float32)
        nodes = np.empty(nn.value, NODE_DTYPE)
        self._lib.orc_export_level(self._h, level, _up(ids), _fp(pts),
                                   nodes.ctypes.data_as(ctypes.c_void_p), ctypes.byref(ns),
                                   ctypes.byref(nn))
        return ids, pts, nodes

    def buffer_pool(self) -> Tuple[np.ndarray, np.ndarray]:
        n = ctypes.c_int64()
        self._lib.orc_export_buffer_pool(self._h, None, None, ctypes.byref(n))
        ids = np.empty(n.value, np.uint32)
        pts = np.empty((n.value, self.dim), np.float32)
        self._lib.orc_export_buffer_pool(self._h, _up(ids), _fp(pts), ctypes.byref(n))
        return ids, pts


def tree_build(pts, ids, leaf_size: int = 16, split: str = "spatial"):
    """BuildvEB over one point set with the spatial or object median; returns
    (pts, ids, nodes, height) with the points in slot order and nodes in vEB
    order."""
    lib = _load()
    p = np.array(pts, dtype=np.float32, copy=True, order="C")
    if p.ndim == 1:
        p = p.reshape(-1, 1)
    d = p.shape[1]
    i = np.array(ids, dtype=np.uint32, copy=True).reshape(-1)
    n = p.shape[0]
    nodes = np.empty(max(1, 2 * n - 1), NODE_DTYPE)
    h = ctypes.c_int32()
    nn = lib.orc_tree_build_rule(d, leaf_size, SPLIT_RULES[split], _fp(p), _up(i), n,
                                 nodes.ctypes.data_as(ctypes.c_void_p), ctypes.byref(h))
    return p, i, nodes[:nn].copy(), h.value


def bruteforce_knn(pts, ids, q, k: int):
    """The definition: k smallest (d2, id) keys over the live points."""
    lib = _load()
    q = np.ascontiguousarray(q, dtype=np.float32)
    d = q.shape[1]
    p = _pts(pts, d)
    i = _ids(ids)
    nq = q.shape[0]
    oi = np.empty((nq, k), np.uint32)
    od = np.empty((nq, k), np.float32)
    lib.orc_bruteforce_knn(d, _fp(p), _up(i), p.shape[0], _fp(q), nq, k, _up(oi), _fp(od))
    return oi, od


def dist2(a, b) -> float:
    lib = _load()
    a = np.ascontiguousarray(a, dtype=np.float32).reshape(-1)
    b = np.ascontiguousarray(b, dtype=np.float32).reshape(-1)
    return float(lib.orc_dist2(a.shape[0], _fp(a), _fp(b)))
