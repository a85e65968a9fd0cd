"""Seeded synthetic inputs for the BDL-tree workloads.

This module is shared by the CPU oracle's tests, the GPU parity tests and the
benchmark.  It only draws numbers: it holds none of the method's arithmetic
(no distances, no splits, no level bookkeeping beyond remembering which ids
are live so that erase batches name live points).

Point sets stand in for the paper's synthetic datasets (Section VI: Uniform
and the clustered VisualVar family); the VisualVar generator itself is not
available, so clustered sets are Gaussian blobs with log-uniform widths and
Zipf-weighted cluster sizes.  All coordinates are float32, ids are uint32.
"""
from __future__ import annotations

import dataclasses
from typing import Iterator, List, Optional, Tuple

import numpy as np

__all__ = [
    "uniform_points",
    "clustered_points",
    "Op",
    "Workload",
    "workload",
    "WORKLOADS",
]


def uniform_points(n: int, d: int, seed: int) -> np.ndarray:
    """n points uniform in [0,1)^d as float32, from PCG64(seed)."""
    rng = np.random.default_rng(seed)
    return rng.random((n, d), dtype=np.float32)


def clustered_points(n: int, d: int, seed: int, n_clusters: int = 100,
                     log10_sigma: Tuple[float, float] = (-4.0, -1.0),
                     zipf_s: float = 1.2, draw_seed: Optional[int] = None) -> np.ndarray:
    """Variable-density clusters: n points from n_clusters Gaussian blobs.

    Centres are uniform in [0,1)^d, each blob's standard deviation is
    10**U(log10_sigma), and blob r (1-based) is chosen with probability
    proportional to r**-zipf_s.  Points are drawn in float64 and cast to
    float32; nothing is clipped.  The mixture comes from `seed`; with
    draw_seed given, the points are drawn from it instead (more points of
    the same mixture).
    """
    rng = np.random.default_rng(seed)
    centres = rng.random((n_clusters, d))
    sigma = 10.0 ** rng.uniform(log10_sigma[0], log10_sigma[1], size=n_clusters)
    w = np.arange(1, n_clusters + 1, dtype=np.float64) ** (-zipf_s)
    w /= w.sum()
    if draw_seed is not None:
        rng = np.random.default_rng(draw_seed)
    which = rng.choice(n_clusters, size=n, p=w)
    out = np.empty((n, d), dtype=np.float32)
    chunk = 1 << 22
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        c = which[s:e]
        z = rng.standard_normal((e - s, d))
        out[s:e] = (centres[c] + sigma[c, None] * z).astype(np.float32)
    return out


@dataclasses.dataclass
class Op:
    """One batch operation: kind is 'insert', 'erase' or 'knn'."""
    kind: str
    pts: np.ndarray                  # [n, d] float32 (points or queries)
    ids: Optional[np.ndarray] = None  # [n] uint32 for insert/erase
    k: int = 0                        # for knn

    @property
    def n(self) -> int:
        return int(self.pts.shape[0])


@dataclasses.dataclass
class Workload:
    name: str
    dim: int
    leaf_size: int
    buffer_size: int
    id_capacity: int
    ops: List[Op]
    description: str = ""
    n_setup: int = 0   # leading ops that only build the resident set


def log_uniform_sizes(rng: np.random.Generator, n: int, lo: float, hi: float) -> np.ndarray:
    """n integer sizes exp(U(ln lo, ln hi)) rounded to nearest, clamped to [lo, hi]."""
    v = np.rint(np.exp(rng.uniform(np.log(lo), np.log(hi), size=n)))
    return np.clip(v, lo, hi).astype(np.int64)


class _LiveIds:
    """Remembers which ids are live (insertion order) to draw erase batches."""

    def __init__(self) -> None:
        self.chunks: List[np.ndarray] = []
        self.dead: Optional[np.ndarray] = None

    def add(self, ids: np.ndarray) -> None:
        self.chunks.append(np.asarray(ids, dtype=np.uint32))

    def live(self) -> np.ndarray:
        allids = np.concatenate(self.chunks) if self.chunks else np.zeros(0, np.uint32)
        if self.dead is not None and self.dead.size:
            allids = allids[~np.isin(allids, self.dead)]
        return allids

    def kill(self, ids: np.ndarray) -> None:
        ids = np.asarray(ids, dtype=np.uint32)
        self.dead = ids if self.dead is None else np.concatenate([self.dead, ids])


def _draw_erase(rng: np.random.Generator, live: np.ndarray, m: int) -> np.ndarray:
    m = min(m, live.size)
    return rng.choice(live, size=m, replace=False).astype(np.uint32)


def _uniform_small(scale: float = 1.0, seed: int = 0, X: int = 1024, d: int = 2) -> Workload:
    """10 inserts of 1000 uniform points, 5 erases of 1000 live points, then
    k=5 queries for 1000 uniform points (leaf 16)."""
    nb = max(1, int(round(1000 * scale)))
    pts = uniform_points(10 * nb, d, seed)
    ids = np.arange(10 * nb, dtype=np.uint32)
    ops: List[Op] = []
    live = _LiveIds()
    for b in range(10):
        sl = slice(b * nb, (b + 1) * nb)
        ops.append(Op("insert", pts[sl], ids[sl]))
        live.add(ids[sl])
    erng = np.random.default_rng(seed + 1)
    for _ in range(5):
        e = _draw_erase(erng, live.live(), nb)
        live.kill(e)
        ops.append(Op("erase", pts[e.astype(np.int64)], e))
    q = uniform_points(max(1, int(round(1000 * scale))), d, seed + 2)
    ops.append(Op("knn", q, k=5))
    return Workload("uniform2d_small", d, 16, X, 10 * nb, ops,
                    "2D uniform, 10x1000 inserts, 5x1000 erases, 1000 queries k=5")


def _uniform3d_10m(scale: float = 1.0, seed: int = 0) -> Workload:
    """Build to n points (10M at scale 1) with 10 equal inserts, erase 10% of
    live ids in one batch, then k=5 queries for every live point in
    ascending id order."""
    d = 3
    n = int(round(10_000_000 * scale))
    nb = n // 10
    n = nb * 10
    pts = uniform_points(n, d, seed)
    ids = np.arange(n, dtype=np.uint32)
    ops: List[Op] = []
    for b in range(10):
        sl = slice(b * nb, (b + 1) * nb)
        ops.append(Op("insert", pts[sl], ids[sl]))
    erng = np.random.default_rng(seed + 1)
    e = np.sort(erng.choice(n, size=nb, replace=False)).astype(np.uint32)
    erng.shuffle(e)
    ops.append(Op("erase", pts[e.astype(np.int64)], e))
    alive = np.ones(n, dtype=bool)
    alive[e.astype(np.int64)] = False
    q = pts[alive]
    ops.append(Op("knn", q, k=5))
    return Workload("uniform3d_10m", d, 16, 1024, n, ops,
                    f"3D uniform, {n} points via 10 inserts of {nb}, erase {nb}, "
                    f"k=5 for all {n - nb} live points")


def _clustered7d(scale: float = 1.0, seed: int = 0) -> Workload:
    """d=7 Gaussian blobs; 100 inserts of n/100, erase 10% in one batch,
    then k=10 for every live point."""
    d = 7
    n = int(round(10_000_000 * scale))
    nb = max(1, n // 100)
    n = nb * 100
    pts = clustered_points(n, d, seed)
    ids = np.arange(n, dtype=np.uint32)
    ops: List[Op] = []
    for b in range(100):
        sl = slice(b * nb, (b + 1) * nb)
        ops.append(Op("insert", pts[sl], ids[sl]))
    erng = np.random.default_rng(seed + 1)
    m = n // 10
    e = erng.choice(n, size=m, replace=False).astype(np.uint32)
    ops.append(Op("erase", pts[e.astype(np.int64)], e))
    alive = np.ones(n, dtype=bool)
    alive[e.astype(np.int64)] = False
    ops.append(Op("knn", pts[alive], k=10))
    return Workload("clustered7d_10m", d, 16, 1024, n, ops,
                    f"7D clustered, {n} points via 100 inserts, erase {m}, k=10 all live")


def _batched5d_20m(scale: float = 1.0, seed: int = 0) -> Workload:
    """Batched-form op log: a 5D uniform resident set of 20M points built by
    20 inserts of 1M (setup), then 4096 kNN batches whose sizes are
    log-uniform in [1, 1e5] with k uniform over {1, 5, 10} and fresh uniform
    queries, and after every 32nd kNN batch one insert of a log-uniform
    [1e3, 1e6] number of fresh uniform points.  `scale` shrinks the resident
    set, the number of kNN batches and the insert sizes together."""
    d = 5
    n_res = int(round(20_000_000 * scale))
    nb = max(1, n_res // 20)
    n_res = nb * 20
    n_knn = max(32, int(round(4096 * scale)))
    rng = np.random.default_rng(seed + 10)
    sizes = log_uniform_sizes(rng, n_knn, 1, max(1, int(round(100_000 * min(1.0, scale * 4)))))
    ks = rng.choice(np.array([1, 5, 10]), size=n_knn)
    n_ins = n_knn // 32
    ins_sizes = log_uniform_sizes(rng, n_ins, max(1, int(1e3 * scale)), max(1, int(1e6 * scale)))
    pts = uniform_points(n_res + int(ins_sizes.sum()), d, seed)
    ids = np.arange(pts.shape[0], dtype=np.uint32)
    q = uniform_points(int(sizes.sum()), d, seed + 20)
    ops: List[Op] = []
    for b in range(20):
        sl = slice(b * nb, (b + 1) * nb)
        ops.append(Op("insert", pts[sl], ids[sl]))
    qo = 0
    po = n_res
    for b in range(n_knn):
        ops.append(Op("knn", q[qo:qo + sizes[b]], k=int(ks[b])))
        qo += int(sizes[b])
        if b % 32 == 31 and b // 32 < n_ins:
            m = int(ins_sizes[b // 32])
            ops.append(Op("insert", pts[po:po + m], ids[po:po + m]))
            po += m
    return Workload("batched5d_20m", d, 16, 1024, int(pts.shape[0]), ops,
                    f"5D uniform, {n_res} resident, {n_knn} kNN batches "
                    f"({int(sizes.sum())} queries, k in {{1,5,10}}), {n_ins} inserts "
                    f"({int(ins_sizes.sum())} points)", n_setup=20)


def _served3d_50m(scale: float = 1.0, seed: int = 0) -> Workload:
    """Served-form request log: a 3D clustered resident set of 50M points
    (the 7D generator's mixture at d=3) built by 50 inserts of 1M (setup),
    then 2000 requests in arrival order: 70% kNN (k=5, log-uniform 1..65536
    fresh queries of the same mixture), 20% inserts (log-uniform 1e3..1e6
    fresh points), 10% erases (log-uniform 1e3..1e6 ids drawn among the live
    ones at that point of the log).  `scale` shrinks every size."""
    d = 3
    n_res = int(round(50_000_000 * scale))
    nb = max(1, n_res // 50)
    n_res = nb * 50
    n_req = max(40, int(round(2000 * min(1.0, scale * 20))))
    rng = np.random.default_rng(seed + 30)
    kinds = rng.choice(np.array(["knn", "insert", "erase"]), size=n_req, p=[0.7, 0.2, 0.1])
    lo, hi = max(1, int(1e3 * scale)), max(2, int(1e6 * scale))
    sizes = {"knn": log_uniform_sizes(rng, n_req, 1, max(2, int(65536 * min(1.0, scale * 20)))),
             "insert": log_uniform_sizes(rng, n_req, lo, hi),
             "erase": log_uniform_sizes(rng, n_req, lo, hi)}
    n_new = int(sum(sizes["insert"][i] for i in range(n_req) if kinds[i] == "insert"))
    pts = clustered_points(n_res + n_new, d, seed)
    ids = np.arange(pts.shape[0], dtype=np.uint32)
    n_q = int(sum(sizes["knn"][i] for i in range(n_req) if kinds[i] == "knn"))
    q = clustered_points(n_q, d, seed, draw_seed=seed + 40)
    alive = np.zeros(pts.shape[0], dtype=bool)
    alive[:n_res] = True
    ops: List[Op] = [Op("insert", pts[b * nb:(b + 1) * nb], ids[b * nb:(b + 1) * nb])
                     for b in range(50)]
    qo, po = 0, n_res
    for i in range(n_req):
        kind = str(kinds[i])
        if kind == "knn":
            m = int(sizes["knn"][i])
            ops.append(Op("knn", q[qo:qo + m], k=5))
            qo += m
        elif kind == "insert":
            m = int(sizes["insert"][i])
            ops.append(Op("insert", pts[po:po + m], ids[po:po + m]))
            alive[po:po + m] = True
            po += m
        else:
            m = int(sizes["erase"][i])
            # draw among the inserted ids, keep live ones (resampling a few
            # times), so that the erase names m live points where possible
            cand = np.unique(rng.integers(0, po, size=int(m * 1.3) + 16))
            cand = cand[alive[cand]]
            rng.shuffle(cand)
            e = cand[:m].astype(np.uint32)
            alive[e.astype(np.int64)] = False
            ops.append(Op("erase", pts[e.astype(np.int64)], e))
    return Workload("served3d_50m", d, 16, 1024, int(pts.shape[0]), ops,
                    f"3D clustered, {n_res} resident, {n_req} requests "
                    f"(70/20/10 kNN/insert/erase), {n_q} queries k=5, {n_new} inserted",
                    n_setup=50)


def _mixed(scale: float = 1.0, seed: int = 0, d: int = 2, clustered: bool = True) -> Workload:
    """The mixed-operations experiment of Section VI-D.3: 20 Insert_L batches
    of 5% of the points each, kNN_L (k = 5) for every live point after every
    fifth insert, then 15 Erase_L batches of 5% each (random live points, no
    repeats) with kNN_L for every live point after every fifth erase: seven
    sections INS0..INS3, DEL0..DEL2.  Points are 10M x scale, clustered
    (the VisualVar stand-in) or uniform; queries are the live points in
    ascending id order."""
    n = int(round(10_000_000 * scale))
    n -= n % 20
    pts = clustered_points(n, d, seed) if clustered else uniform_points(n, d, seed)
    ids = np.arange(n, dtype=np.uint32)
    b = n // 20
    ops: List[Op] = []
    for i in range(20):
        ops.append(Op("insert", pts[i * b:(i + 1) * b], ids[i * b:(i + 1) * b]))
        if i % 5 == 4:
            ops.append(Op("knn", pts[:(i + 1) * b], k=5))
    order = np.random.default_rng(seed + 1).permutation(n)
    alive = np.ones(n, bool)
    for i in range(15):
        e = np.sort(order[i * b:(i + 1) * b])
        alive[e] = False
        ops.append(Op("erase", pts[e], ids[e]))
        if i % 5 == 4:
            ops.append(Op("knn", pts[alive], k=5))
    kind = "clustered" if clustered else "uniform"
    return Workload(f"mixed{d}d_10m", d, 16, 1024, n, ops,
                    f"{d}D {kind} {n} points: 20 inserts of {b}, 15 erases of {b}, "
                    f"kNN_L k=5 of every live point after every 5 updates")


WORKLOADS = {
    "uniform2d_small": _uniform_small,
    "served3d_50m": _served3d_50m,
    "batched5d_20m": _batched5d_20m,
    "uniform3d_10m": _uniform3d_10m,
    "clustered7d_10m": _clustered7d,
    "mixed2d_10m": lambda scale=1.0, seed=0: _mixed(scale, seed, d=2, clustered=True),
    "mixed7d_10m": lambda scale=1.0, seed=0: _mixed(scale, seed, d=7, clustered=False),
}


def workload(name: str, scale: float = 1.0, seed: int = 0, **kw) -> Workload:
    return WORKLOADS[name](scale=scale, seed=seed, **kw)


def random_op_sequence(seed: int, d: int, n_ops: int, max_batch: int,
                       id_capacity: int, p_insert: float = 0.5,
                       p_erase: float = 0.3, clustered: bool = False,
                       k_max: int = 16, bad_erase_frac: float = 0.1) -> Iterator[Op]:
    """Random interleaved inserts, erases and queries for stress tests.

    Erase batches mostly name live (id, point) pairs; a fraction names ids
    that are not live, or live ids with perturbed coordinates, or repeats an
    id inside the batch.  Ids are drawn without reuse from [0, id_capacity).
    """
    rng = np.random.default_rng(seed)
    next_id = 0
    live_ids: List[int] = []
    store = {}
    for _ in range(n_ops):
        r = rng.random()
        if r < p_insert or not live_ids:
            b = int(rng.integers(0, max_batch + 1))
            b = min(b, id_capacity - next_id)
            if clustered:
                p = clustered_points(b, d, int(rng.integers(1 << 30)), n_clusters=4)
            else:
                p = rng.random((b, d), dtype=np.float32)
            # occasional exact duplicates of coordinates (distinct ids)
            if b > 4 and rng.random() < 0.3:
                src = rng.integers(0, b, size=b // 4)
                dst = rng.integers(0, b, size=b // 4)
                p[dst] = p[src]
            ids = np.arange(next_id, next_id + b, dtype=np.uint32)
            next_id += b
            for i in range(b):
                store[int(ids[i])] = p[i].copy()
            live_ids.extend(int(x) for x in ids)
            yield Op("insert", p, ids)
        elif r < p_insert + p_erase:
            b = int(rng.integers(0, min(max_batch, len(live_ids)) + 1))
            pick = rng.choice(len(live_ids), size=b, replace=False) if b else np.zeros(0, np.int64)
            ids = [live_ids[i] for i in pick]
            pts = [store[i].copy() for i in ids]
            nbad = int(round(bad_erase_frac * b))
            for j in range(nbad):
                kind = rng.integers(0, 3)
                if kind == 0:       # id never inserted
                    ids.append(int(next_id + rng.integers(0, 1000)))
                    pts.append(rng.random(d, dtype=np.float32))
                elif kind == 1:     # live id, wrong coordinates
                    i = live_ids[int(rng.integers(0, len(live_ids)))]
                    p = store[i].copy()
                    p[int(rng.integers(0, d))] += np.float32(0.25)
                    ids.append(i)
                    pts.append(p)
                else:               # repeat an id already in the batch
                    if ids:
                        j2 = int(rng.integers(0, len(ids)))
                        ids.append(ids[j2])
                        pts.append(pts[j2].copy())
            killed = set(live_ids[i] for i in pick)
            live_ids = [i for i in live_ids if i not in killed]
            arr = np.array(pts, dtype=np.float32).reshape(-1, d)
            yield Op("erase", arr, np.array(ids, dtype=np.uint32))
        else:
            nq = int(rng.integers(0, max_batch + 1))
            q = rng.random((nq, d), dtype=np.float32)
            if live_ids and nq > 2:
                # some queries sit exactly on live points
                for j in range(0, nq, 3):
                    q[j] = store[live_ids[int(rng.integers(0, len(live_ids)))]]
            k = int(rng.integers(1, k_max + 1))
            yield Op("knn", q, k=k)
