"""The k-NN graph (bdl_knn_graph) against the oracle's kNN_L on the GPU.

bdl_knn_graph answers kNN_L (Alg. 5) for every live point, either from
presorted queries searched from the roots or started from each point's own
subtree (BDL_PARAM_GRAPH_START).  In both ways its row `id` must equal, id
for id and distance bit for bit, the oracle's kNN_L row for live point `id`
as a query; rows of ids that are not live stay untouched.  The cases cover tombstones and the buffer,
leaves larger than a wavefront (leaf size 128, and B2's grown leaves),
coincident points, both split rules, k from 1 to 64 and dimensions 1 to 16.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from bdl_inputs import Op, clustered_points, random_op_sequence, uniform_points
from gpu_util import assert_knn_equal, bits, log, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    t.cuda.set_device(0)
    return t


@pytest.fixture(scope="module")
def bdl():
    import paper_2112_06188_amd as m
    m.load_library()
    return m


def live_points(o):
    """(ids ascending, points) of every live point the oracle holds."""
    ids, pts = [], []
    for j in bits(o.level_info()["F"]):
        i, p, _ = o.export_level(j)
        ids.append(i)
        pts.append(p)
    i, p = o.buffer_pool()
    ids.append(i)
    pts.append(p)
    ids = np.concatenate(ids)
    pts = np.concatenate(pts).reshape(len(ids), o.dim)
    keep = ids != np.uint32(0xFFFFFFFF)
    ids, pts = ids[keep], pts[keep]
    order = np.argsort(ids, kind="stable")
    return ids[order], pts[order]


def check_graph(t, o, k, what):
    """Both ways to the graph (presorted queries from the roots, and the
    leaf-based search) against the oracle's kNN_L over the live points."""
    import paper_2112_06188_amd as bdl
    ids, pts = live_points(o)
    assert len(ids) == o.size() == t.size(), what
    oi = od = None
    if len(ids):
        oi, od = o.knn(pts, k)
    for start in (0, 1):
        t.set_param(bdl.PARAM_GRAPH_START, start)
        gi, gd = t.knn_graph(k)
        t.sync()
        gi = gi.cpu().numpy().view(np.uint32)
        gd = gd.cpu().numpy()
        tag = f"{what} start={start}"
        if len(ids):
            assert_knn_equal(gi[ids.astype(np.int64)], gd[ids.astype(np.int64)], oi, od, tag)
        dead = np.ones(gi.shape[0], bool)
        dead[ids.astype(np.int64)] = False
        assert (gi[dead] == np.uint32(0xFFFFFFFF)).all(), f"{tag}: a row of a dead id was written"
        assert np.isinf(gd[dead]).all(), tag
    t.set_param(bdl.PARAM_GRAPH_START, 0)


@pytest.mark.parametrize("seed,d,leaf,X,k,clustered,split", [
    (0, 2, 4, 64, 5, False, "spatial"), (1, 3, 16, 128, 10, True, "spatial"),
    (2, 7, 8, 32, 1, True, "object"), (3, 1, 2, 16, 17, False, "spatial"),
    (4, 16, 16, 64, 64, False, "object"), (5, 5, 128, 256, 8, True, "spatial"),
    (6, 3, 1, 8, 3, False, "spatial"),
])
def test_graph_random_ops(torch, bdl, seed, d, leaf, X, k, clustered, split):
    log(f"case: knn graph seed={seed} d={d} leaf={leaf} X={X} k={k} {split}")
    idcap = 1 << 16
    t = bdl.Tree(d, leaf_size=leaf, buffer_size=X, id_capacity=idcap, split=split)
    o = oracle.OracleBDL(d, leaf, X, split=split)
    ops = [op for op in random_op_sequence(200 + seed, d, n_ops=24, max_batch=600,
                                           id_capacity=idcap, clustered=clustered)
           if op.kind != "knn"]
    for n_op, op in enumerate(ops):
        if op.kind == "insert":
            t.insert(to_dev(op.pts, torch), to_dev(op.ids, torch))
            o.insert(op.pts, op.ids)
        else:
            assert t.erase(to_dev(op.pts, torch), to_dev(op.ids, torch)) == o.erase(op.pts, op.ids)
        if n_op % 6 == 5:
            check_graph(t, o, k, f"graph seed={seed} op{n_op}")
    check_graph(t, o, k, f"graph seed={seed} final")
    t.close()


def test_graph_empty_and_tiny(torch, bdl):
    log("case: knn graph empty and tiny")
    d = 3
    t = bdl.Tree(d, leaf_size=16, buffer_size=64, id_capacity=100)
    o = oracle.OracleBDL(d, 16, 64)
    check_graph(t, o, 5, "empty")
    p = uniform_points(3, d, 1)
    ids = np.array([7, 3, 99], np.uint32)
    t.insert(to_dev(p, torch), to_dev(ids, torch))
    o.insert(p, ids)
    check_graph(t, o, 5, "three points in the buffer")
    t.close()


def test_graph_coincident_points(torch, bdl):
    """Many copies of few points: degenerate leaves far larger than 64."""
    log("case: knn graph coincident")
    d = 2
    base = uniform_points(5, d, 3)
    p = np.repeat(base, 400, axis=0)
    ids = np.random.default_rng(4).permutation(len(p)).astype(np.uint32)
    t = bdl.Tree(d, leaf_size=16, buffer_size=256, id_capacity=len(p))
    o = oracle.OracleBDL(d, 16, 256)
    t.insert(to_dev(p, torch), to_dev(ids, torch))
    o.insert(p, ids)
    check_graph(t, o, 7, "coincident")
    t.close()


@pytest.mark.parametrize("structure", ["rebuild_all", "no_rebuild"])
def test_graph_baselines(torch, bdl, structure):
    """B2's leaves grow far past the leaf size while the nodes keep the
    point counts of the first build; the groups must still cover every
    slot once."""
    log(f"case: knn graph {structure}")
    d = 3
    t = bdl.Tree(d, leaf_size=16, buffer_size=64, id_capacity=1 << 17, structure=structure)
    o = oracle.OracleBDL(d, 16, 64, mode=structure)
    base = uniform_points(20_000, d, 30)
    hot = clustered_points(40_000, d, 31, n_clusters=1, log10_sigma=(-2.5, -2.5))
    ids = np.arange(60_000, dtype=np.uint32)
    for op in [Op("insert", base, ids[:20_000]), Op("insert", hot[:20_000], ids[20_000:40_000]),
               Op("erase", base[::3], ids[:20_000:3]), Op("insert", hot[20_000:], ids[40_000:])]:
        if op.kind == "insert":
            t.insert(to_dev(op.pts, torch), to_dev(op.ids, torch))
            o.insert(op.pts, op.ids)
        else:
            assert t.erase(to_dev(op.pts, torch), to_dev(op.ids, torch)) == o.erase(op.pts, op.ids)
    check_graph(t, o, 6, structure)
    t.close()


def test_graph_equals_knn_at_scale(torch, bdl):
    """2M uniform 3D points in 10 batches and an erase of a tenth: the graph
    equals kNN_L over every live point (queries in id order) bit for bit,
    and sampled rows equal the oracle's."""
    log("case: knn graph 2M")
    d, n, k = 3, 2_000_000, 5
    pts = uniform_points(n, d, 40)
    ids = np.arange(n, dtype=np.uint32)
    dp, di = to_dev(pts, torch), to_dev(ids, torch)
    t = bdl.Tree(d, leaf_size=16, buffer_size=1024, id_capacity=n)
    for s in range(0, n, n // 10):
        t.insert(dp[s:s + n // 10], di[s:s + n // 10])
    e = np.sort(np.random.default_rng(41).choice(n, n // 10, replace=False))
    ed = torch.from_numpy(e).cuda()
    assert t.erase(dp[ed], di[ed]) == len(e)
    live = np.ones(n, bool)
    live[e] = False
    lid = np.flatnonzero(live)
    ld = torch.from_numpy(lid).cuda()
    qi, qd = t.knn(dp[ld], k)
    sel = lid[np.random.default_rng(42).choice(len(lid), 64, replace=False)]
    oi, od = oracle.bruteforce_knn(pts[live], lid.astype(np.uint32), pts[sel], k)
    for start in (0, 1):
        t.set_param(bdl.PARAM_GRAPH_START, start)
        gi, gd = t.knn_graph(k)
        t.sync()
        assert torch.equal(gi[ld], qi), f"start={start}: graph ids differ from kNN_L"
        assert torch.equal(gd[ld].view(torch.int32), qd.view(torch.int32)), \
            f"start={start}: graph distances differ from kNN_L"
        assert_knn_equal(gi.cpu().numpy()[sel], gd.cpu().numpy()[sel], oi, od,
                         f"graph 2M sampled start={start}")
    t.close()
