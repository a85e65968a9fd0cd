"""Insert_L without host waits.

bdl_insert enqueues the whole insert (gather, every build depth the data
needs, the LDS finisher, the vEB layout) on the tree's stream: a sequence of
inserts into a tree whose scratch is already large enough blocks the host
zero times, counted by bdl_host_waits.  Clustered points need far more build
depths than log2(n / finisher size), which used to cost a host round trip per
extra budget of depths.  Afterwards the structure and the k-NN rows must
equal the oracle's.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from bdl_inputs import clustered_points, uniform_points
from gpu_util import assert_knn_equal, compare_structure, log, to_dev

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


@pytest.mark.parametrize("d,clustered,split", [(3, False, "spatial"), (7, True, "spatial"),
                                               (3, True, "object"), (2, True, "spatial")])
def test_ten_inserts_without_host_waits(torch, bdl, d, clustered, split):
    log(f"case: async inserts d={d} clustered={clustered} split={split}")
    n, b = 600_000, 60_000
    pts = clustered_points(n, d, 40 + d, log10_sigma=(-4.0, -1.0)) if clustered \
        else uniform_points(n, d, 40 + d)
    ids = np.arange(n, dtype=np.uint32)
    dp, di = to_dev(pts, torch), to_dev(ids, torch)
    t = bdl.Tree(d, leaf_size=16, buffer_size=1024, id_capacity=n, split=split)
    # first pass grows the scratch and the arenas to their final sizes
    for s in range(0, n, b):
        t.insert(dp[s:s + b], di[s:s + b])
    t.sync()
    t.clear()
    t.sync()
    w0 = t.host_waits()
    for s in range(0, n, b):
        t.insert(dp[s:s + b], di[s:s + b])
    assert t.host_waits() == w0, "an insert blocked the host"
    t.sync()
    o = oracle.OracleBDL(d, 16, 1024, split=split)
    for s in range(0, n, b):
        o.insert(pts[s:s + b], ids[s:s + b])
    compare_structure(t, o, d, f"async d={d}")
    q = np.concatenate([pts[::397], uniform_points(1000, d, 7)]).astype(np.float32)
    gi, gd = t.knn(to_dev(q, torch), 8)
    t.sync()
    oi, od = o.knn(q, 8)
    assert_knn_equal(gi.cpu().numpy(), gd.cpu().numpy(), oi, od, f"async knn d={d}")
    t.close()


def test_inserts_and_queries_interleave_without_waits(torch, bdl):
    """k-NN launches between inserts read the trees' node counts on the
    device: results equal the oracle's at every step, with no wait until the
    final readback."""
    log("case: async inserts interleaved with k-NN")
    d, n, b = 3, 200_000, 25_000
    pts = uniform_points(n, d, 50)
    ids = np.arange(n, dtype=np.uint32)
    dp, di = to_dev(pts, torch), to_dev(ids, torch)
    t = bdl.Tree(d, leaf_size=16, buffer_size=1024, id_capacity=n)
    for s in range(0, n, b):
        t.insert(dp[s:s + b], di[s:s + b])
    t.sync()
    t.clear()
    t.sync()
    q = uniform_points(3000, d, 51)
    dq = to_dev(q, torch)
    w0 = t.host_waits()
    outs = []
    for s in range(0, n, b):
        t.insert(dp[s:s + b], di[s:s + b])
        outs.append(t.knn(dq, 5))
    assert t.host_waits() == w0
    t.sync()
    o = oracle.OracleBDL(d, 16, 1024)
    for j, s in enumerate(range(0, n, b)):
        o.insert(pts[s:s + b], ids[s:s + b])
        oi, od = o.knn(q, 5)
        assert_knn_equal(outs[j][0].cpu().numpy(), outs[j][1].cpu().numpy(), oi, od,
                         f"step {j}")
    t.close()
