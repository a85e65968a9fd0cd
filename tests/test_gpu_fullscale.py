"""The batched and served forms at (near) full scale.

- Batched: the full 20M-point 5D resident set of the batched op log and its
  first 256 kNN batches (with the inserts among them): the batched calls
  give the plain per-call results bit for bit, and two rows of every batch
  equal the brute-force definition over the points live at that time.
- Served: the served request log at a fifth of its size (10M resident 3D
  clustered points, 2000 requests): every result equals a plain replay in
  admission order, erase counts included.
"""
from __future__ import annotations

import time

import numpy as np
import pytest

import oracle
from bdl_inputs import workload
from gpu_util import assert_knn_equal, log, to_dev

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


def test_batched5d_20m_full_slice(torch, bdl):
    w = workload("batched5d_20m")
    log(f"case: batched op log full resident set, first 256 batches: {w.description}")
    trees = [bdl.Tree(w.dim, leaf_size=w.leaf_size, buffer_size=w.buffer_size,
                      id_capacity=w.id_capacity) for _ in range(2)]
    for op in w.ops[:w.n_setup]:
        dp, di = to_dev(op.pts, torch), to_dev(op.ids, torch)
        for t in trees:
            t.insert(dp, di)
    live_pts = [op.pts for op in w.ops[:w.n_setup]]
    live_ids = [op.ids for op in w.ops[:w.n_setup]]
    rng = np.random.default_rng(11)
    plain, batched, pend, checks = [], [], [], []

    def flush():
        if pend:
            batched.extend(trees[1].knn_batch([(to_dev(q, torch), k) for q, k in pend]))
            pend.clear()

    def brute():
        # the rows chosen since the last insert, against the points live for
        # them: one brute-force pass per k
        todo = [c for c in checks if c[3] is None]
        if not todo:
            return
        P = np.concatenate(live_pts)
        I = np.concatenate(live_ids)
        for k in sorted({c[2] for c in todo}):
            part = [c for c in todo if c[2] == k]
            oi, od = oracle.bruteforce_knn(P, I, np.concatenate([c[1] for c in part]), k)
            at = 0
            for c in part:
                m = c[1].shape[0]
                c[3] = (oi[at:at + m], od[at:at + m])
                at += m

    n_knn = 0
    for op in w.ops[w.n_setup:]:
        if op.kind == "knn":
            if n_knn == 256:
                break
            n_knn += 1
            plain.append(trees[0].knn(to_dev(op.pts, torch), op.k))
            pend.append((op.pts, op.k))
            rows = rng.choice(op.n, size=min(2, op.n), replace=False)
            checks.append([len(plain) - 1, op.pts[rows], op.k, None, rows])
        else:
            flush()
            brute()
            for t in trees:
                t.insert(to_dev(op.pts, torch), to_dev(op.ids, torch))
            live_pts.append(op.pts)
            live_ids.append(op.ids)
    flush()
    brute()
    for t in trees:
        t.sync()
    assert len(plain) == len(batched) == 256
    for (pi, pd), (bi, bd) in zip(plain, batched):
        assert torch.equal(pi, bi) and torch.equal(pd.view(torch.int32), bd.view(torch.int32))
    for j, q, k, (oi, od), rows in checks:
        bi, bd = batched[j]
        assert_knn_equal(bi.cpu().numpy()[rows], bd.cpu().numpy()[rows], oi, od, f"batch {j}")
    for t in trees:
        t.close()


def test_served3d_log_at_scale_0_2(torch, bdl):
    w = workload("served3d_50m", scale=0.2)
    log(f"case: served log at scale 0.2: {w.description}")
    mk = lambda: bdl.Tree(w.dim, leaf_size=w.leaf_size, buffer_size=w.buffer_size,
                          id_capacity=w.id_capacity)
    t, r = mk(), mk()
    for op in w.ops[:w.n_setup]:
        dp, di = to_dev(op.pts, torch), to_dev(op.ids, torch)
        t.insert(dp, di)
        r.insert(dp, di)
    t.sync()
    srv = bdl.Server(t, mode=1, max_inflight=256, mem_budget=2 << 30)
    reqs = w.ops[w.n_setup:]
    at = np.cumsum(np.random.default_rng(5).exponential(1.0 / 1000.0, size=len(reqs)))
    t0 = time.perf_counter()
    tickets = []
    for a, op in zip(at, reqs):
        while time.perf_counter() < t0 + a:
            pass
        if op.kind == "knn":
            tickets.append(srv.submit_knn(op.pts, op.k))
        elif op.kind == "insert":
            tickets.append(srv.submit_insert(op.pts, op.ids))
        else:
            tickets.append(srv.submit_erase(op.pts, op.ids))
    comps = [srv.wait(tk) for tk in tickets]
    srv.close()
    log(f"served {len(comps)} requests in {time.perf_counter() - t0:.1f} s")
    order = np.argsort([c["admit_seq"] for c in comps])
    assert [comps[i]["admit_seq"] for i in order] == list(range(len(comps)))
    for j, i in enumerate(order):
        c, op = comps[i], reqs[i]
        assert c["status"] == 0, j
        if op.kind == "insert":
            r.insert(to_dev(op.pts, torch), to_dev(op.ids, torch))
        elif op.kind == "erase":
            assert r.erase(to_dev(op.pts, torch), to_dev(op.ids, torch)) == c["n_erased"], j
        else:
            gi, gd = r.knn(to_dev(op.pts, torch), op.k)
            r.sync()
            assert np.array_equal(gi.cpu().numpy().view(np.uint32), c["ids"]), j
            assert np.array_equal(gd.cpu().numpy().view(np.uint32), c["d2"].view(np.uint32)), j
    assert t.size() == r.size()
    t.close()
    r.close()
