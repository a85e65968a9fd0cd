"""The batched form of kNN_L (bdl_knn_batch): many requests of uneven size
and different k in one launch sequence, replayed from captured hipGraphs.

Its results must be those of the plain per-call path bit for bit, and the
oracle's.  Graph replays are checked several times in a row, with eager work,
synchronisations and tree updates in between, against eager results.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from bdl_inputs import uniform_points
from gpu_util import assert_knn_equal, log, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    t.cuda.set_device(0)
    return t


@pytest.fixture(scope="module")
def bdl():
    import paper_2112_06188_amd as m
    m.load_library()
    return m


def _requests(rng, d, n_req, max_n, ks):
    reqs = []
    for _ in range(n_req):
        n = int(np.exp(rng.uniform(0, np.log(max_n))))
        reqs.append((uniform_points(n, d, int(rng.integers(1 << 30))), int(rng.choice(ks))))
    return reqs


@pytest.mark.parametrize("graphs", [1, 0])
@pytest.mark.parametrize("kern", [1, 0])
def test_batch_equals_plain_and_oracle(torch, bdl, graphs, kern):
    log(f"case: batch graphs={graphs} kernel={kern}")
    d = 3
    t = bdl.Tree(d, leaf_size=16, buffer_size=256, id_capacity=1 << 20)
    t.set_param(bdl.PARAM_USE_GRAPHS, graphs)
    t.set_param(bdl.PARAM_KNN_KERNEL, kern)
    o = oracle.OracleBDL(d, 16, 256)
    p = uniform_points(60_000, d, 3)
    ids = np.arange(60_000, dtype=np.uint32)
    t.insert(to_dev(p, torch), to_dev(ids, torch))
    o.insert(p, ids)
    rng = np.random.default_rng(4)
    for ks in ([1, 5, 10], [1, 2], [7, 17, 3], [33, 64, 5]):
        reqs = _requests(rng, d, 25, 20_000, ks)
        reqs.append((uniform_points(0, d, 1), 5))          # an empty request
        outs = t.knn_batch([(to_dev(q, torch), k) for q, k in reqs])
        t.sync()
        for (q, k), (gi, gd) in zip(reqs, outs):
            if len(q) == 0:
                continue
            pi, pd = t.knn(to_dev(q, torch), k)
            t.sync()
            assert torch.equal(gi, pi) and torch.equal(gd.view(torch.int32), pd.view(torch.int32))
            sel = slice(0, min(len(q), 300))
            oi, od = o.knn(q[sel], k)
            assert_knn_equal(gi.cpu().numpy()[sel], gd.cpu().numpy()[sel], oi, od, f"k={k}")
    t.close()


def test_graph_replays_across_updates(torch, bdl):
    """One size bucket replayed many times; between replays the tree changes
    (inserts, erases with rebuilds), plain eager queries run and the stream is
    synchronised.  Every replay matches the oracle at that moment."""
    log("case: graph replays")
    d = 2
    X = 64
    t = bdl.Tree(d, leaf_size=8, buffer_size=X, id_capacity=1 << 20)
    o = oracle.OracleBDL(d, 8, X)
    rng = np.random.default_rng(5)
    nid = 0
    live = {}
    for rnd in range(8):
        n = int(rng.integers(500, 6000))
        p = uniform_points(n, d, 100 + rnd)
        ids = np.arange(nid, nid + n, dtype=np.uint32)
        nid += n
        t.insert(to_dev(p, torch), to_dev(ids, torch))
        o.insert(p, ids)
        for i, q in zip(ids, p):
            live[int(i)] = q
        if rnd % 2 == 1:
            e = rng.choice(np.array(sorted(live), dtype=np.uint32), size=len(live) // 3,
                           replace=False)
            ep = np.array([live[int(i)] for i in e], np.float32)
            assert t.erase(to_dev(ep, torch), to_dev(e, torch)) == o.erase(ep, e)
            for i in e:
                del live[int(i)]
        # same bucket (<= 4096 queries in all) every round
        reqs = [(uniform_points(int(rng.integers(1, 900)), d, 1000 + rnd * 10 + j),
                 int(rng.choice([1, 5, 10]))) for j in range(4)]
        outs = t.knn_batch([(to_dev(q, torch), k) for q, k in reqs])
        # eager work and a synchronisation between replays
        eq = uniform_points(300, d, 2000 + rnd)
        ei, ed = t.knn(to_dev(eq, torch), 4)
        t.sync()
        oi, od = o.knn(eq, 4)
        assert_knn_equal(ei.cpu().numpy(), ed.cpu().numpy(), oi, od, f"eager rnd={rnd}")
        for (q, k), (gi, gd) in zip(reqs, outs):
            oi, od = o.knn(q, k)
            assert_knn_equal(gi.cpu().numpy(), gd.cpu().numpy(), oi, od, f"replay rnd={rnd}")
    t.close()


def test_batched_oplog_matches_plain_and_oracle(torch, bdl):
    """The batched-form op log (5D, uneven kNN batches with k in {1,5,10},
    an insert after every 32nd batch) at reduced scale: the batched calls
    (one per run of kNN batches between inserts) give the plain per-call
    results bit for bit, and the oracle's on the first rows of every batch."""
    from bdl_inputs import workload
    w = workload("batched5d_20m", scale=0.02)
    log(f"case: batched op log: {w.description}")
    trees = [bdl.Tree(w.dim, leaf_size=w.leaf_size, buffer_size=w.buffer_size,
                      id_capacity=w.id_capacity) for _ in range(2)]
    o = oracle.OracleBDL(w.dim, w.leaf_size, w.buffer_size)
    for op in w.ops[:w.n_setup]:
        for t in trees:
            t.insert(to_dev(op.pts, torch), to_dev(op.ids, torch))
        o.insert(op.pts, op.ids)
    plain, batched, pend = [], [], []

    def flush():
        if pend:
            batched.extend(trees[1].knn_batch([(to_dev(q, torch), k) for q, k in pend]))
            pend.clear()

    for op in w.ops[w.n_setup:]:
        if op.kind == "knn":
            plain.append(trees[0].knn(to_dev(op.pts, torch), op.k))
            pend.append((op.pts, op.k))
            oi, od = o.knn(op.pts[:16], op.k)
            plain[-1] = plain[-1] + ((oi, od),)
        else:
            flush()
            for t in trees:
                t.insert(to_dev(op.pts, torch), to_dev(op.ids, torch))
            o.insert(op.pts, op.ids)
    flush()
    for t in trees:
        t.sync()
    assert len(plain) == len(batched)
    for (pi, pd, (oi, od)), (bi, bd) in zip(plain, batched):
        assert torch.equal(pi, bi) and torch.equal(pd.view(torch.int32), bd.view(torch.int32))
        assert_knn_equal(bi.cpu().numpy()[:16], bd.cpu().numpy()[:16], oi, od, "batched op log")
    for t in trees:
        t.close()
