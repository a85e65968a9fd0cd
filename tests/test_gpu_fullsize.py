"""The 10M-point 3D workload at full size, in the launch configuration the
benchmark times: 10 Insert_L batches of 1M uniform points, one Erase_L of
1M random live points, kNN_L k=5 for all 9M live points.

Checked at full size: every tree (slot order, points, node arrays) against
the oracle's after the inserts and again after the erase, the level
schedule against the binary-counter closed form, the self-match property
for every query (each query is a live point and coordinates are distinct,
so its nearest neighbour is itself at 0), and sampled rows against the
brute-force definition over the live set.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from bdl_inputs import workload
from gpu_util import assert_knn_equal, bits, compare_structure, log, to_dev

pytestmark = pytest.mark.gpu


def test_uniform3d_10m_full_size():
    import torch

    import paper_2112_06188_amd as bdl

    torch.cuda.set_device(0)
    log("case: uniform3d_10m full size")
    w = workload("uniform3d_10m")
    t = bdl.Tree(w.dim, leaf_size=w.leaf_size, buffer_size=w.buffer_size,
                 id_capacity=w.id_capacity)
    o = oracle.OracleBDL(w.dim, w.leaf_size, w.buffer_size)
    live = np.ones(w.id_capacity, dtype=bool)
    all_pts = np.concatenate([op.pts for op in w.ops if op.kind == "insert"])
    for op in w.ops:
        if op.kind == "insert":
            t.insert(to_dev(op.pts, torch), to_dev(op.ids, torch))
            o.insert(op.pts, op.ids)
        elif op.kind == "erase":
            # before the erase: the closed form of 10M insert-only points
            info = t.level_info()
            assert bits(info["F"]) == [0, 2, 5, 9, 10, 13] and info["buf_live"] == 640
            compare_structure(t, o, w.dim, "10M after the inserts")
            assert t.erase(to_dev(op.pts, torch), to_dev(op.ids, torch)) == op.n
            assert o.erase(op.pts, op.ids) == op.n
            live[op.ids.astype(np.int64)] = False
            compare_structure(t, o, w.dim, "10M after the erase")
        else:
            qop = op
    o.close()
    info = t.level_info()
    assert bits(info["F"]) == [0, 2, 5, 9, 10, 13]
    # the buffer holds the 640 newest points and loses those the erase names
    assert info["buf_live"] == int(live[w.id_capacity - 640:].sum())
    assert t.counters()["rebuilt"] == 23_520_256
    # erasing 10% uniformly keeps every tree above half capacity
    assert t.counters()["reinserted"] == 0
    assert t.size() == 9_000_000
    gi, gd = t.knn(to_dev(qop.pts, torch), qop.k)
    t.sync()
    qids = np.nonzero(live)[0].astype(np.uint32)
    assert torch.equal(gi[:, 0], to_dev(qids, torch))
    assert bool((gd[:, 0] == 0).all())
    assert bool((gd[:, 1:] >= gd[:, :-1]).all())
    rng = np.random.default_rng(7)
    sel = np.sort(rng.choice(qop.n, size=192, replace=False))
    oi, od = oracle.bruteforce_knn(all_pts[live], qids, qop.pts[sel], qop.k)
    assert_knn_equal(gi.cpu().numpy()[sel], gd.cpu().numpy()[sel], oi, od, "full size sample")
    t.close()


def test_clustered7d_10m_full_size():
    """The 7D clustered workload at full size: 100 Insert_L batches of 100K,
    one Erase_L of 1M live ids, kNN_L k=10 for every live point.  Checked:
    the schedule against the binary-counter closed form (insert-only up to
    the erase), the half rule after the erase, the self-match property where
    coordinates are unique, and sampled rows against brute force."""
    import torch

    import paper_2112_06188_amd as bdl

    torch.cuda.set_device(0)
    log("case: clustered7d_10m full size")
    w = workload("clustered7d_10m")
    t = bdl.Tree(w.dim, leaf_size=w.leaf_size, buffer_size=w.buffer_size,
                 id_capacity=w.id_capacity)
    live = np.ones(w.id_capacity, dtype=bool)
    all_pts = np.concatenate([op.pts for op in w.ops if op.kind == "insert"])
    n = len(all_pts)
    for op in w.ops:
        if op.kind == "insert":
            t.insert(to_dev(op.pts, torch), to_dev(op.ids, torch))
        elif op.kind == "erase":
            info = t.level_info()
            m = n // w.buffer_size
            assert info["F"] == m and info["buf_live"] == n - m * w.buffer_size
            assert t.erase(to_dev(op.pts, torch), to_dev(op.ids, torch)) == op.n
            live[op.ids.astype(np.int64)] = False
        else:
            qop = op
    info = t.level_info()
    cap = info["cap"]
    for i in bits(info["F"]):
        assert 2 * info["live"][i] >= cap[i], f"tree {i} below half after the erase"
    assert t.size() == int(live.sum())
    gi, gd = t.knn(to_dev(qop.pts, torch), qop.k)
    t.sync()
    qids = np.nonzero(live)[0].astype(np.uint32)
    # a query whose coordinates occur once among the live points finds
    # itself first at distance 0
    _, first, counts = np.unique(qop.pts, axis=0, return_index=True, return_counts=True)
    uniq = np.zeros(len(qids), dtype=bool)
    uniq[first[counts == 1]] = True
    g0 = gi[:, 0].cpu().numpy().view(np.uint32)
    assert np.array_equal(g0[uniq], qids[uniq])
    assert bool((gd[:, 0] == 0).all())
    assert bool((gd[:, 1:] >= gd[:, :-1]).all())
    rng = np.random.default_rng(8)
    sel = np.sort(rng.choice(qop.n, size=160, replace=False))
    oi, od = oracle.bruteforce_knn(all_pts[live], qids, qop.pts[sel], qop.k)
    assert_knn_equal(gi.cpu().numpy()[sel], gd.cpu().numpy()[sel], oi, od, "7D full size sample")
    t.close()


def test_one_build_with_a_long_node_list():
    """One Insert_L of 2^14 * 1200 uniform 3D points builds a single tree
    whose deepest global depth lists about 8192 nodes, more than the list
    kernel keeps in LDS, so the next depth's tiles are found through the
    device copy of the tile starts.  Checked: the level schedule, the size,
    self-matches and sampled rows against brute force."""
    import torch

    import paper_2112_06188_amd as bdl
    from bdl_inputs import uniform_points

    torch.cuda.set_device(0)
    log("case: one build with a long node list")
    d, X = 3, 1200
    n = (1 << 14) * X
    pts = uniform_points(n, d, 11)
    ids = np.arange(n, dtype=np.uint32)
    t = bdl.Tree(d, leaf_size=16, buffer_size=X, id_capacity=n)
    t.insert(to_dev(pts, torch), to_dev(ids, torch))
    info = t.level_info()
    assert bits(info["F"]) == [14] and info["buf_live"] == 0
    assert t.size() == n
    rng = np.random.default_rng(12)
    sel = np.sort(rng.choice(n, size=64, replace=False))
    q = np.concatenate([pts[sel], uniform_points(64, d, 13)]).astype(np.float32)
    gi, gd = t.knn(to_dev(q, torch), 8)
    t.sync()
    assert torch.equal(gi[:64, 0], to_dev(ids[sel], torch))
    oi, od = oracle.bruteforce_knn(pts, ids, q, 8)
    assert_knn_equal(gi.cpu().numpy(), gd.cpu().numpy(), oi, od, "long node list")
    t.close()
