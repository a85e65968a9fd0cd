"""Parity of the HIP library with the CPU oracle on the GPU.

Every case runs the same operations on both, then compares exactly: the
static trees (slot order, points, node arrays in vEB order), the buffer, the
live counts and every k-NN row (ids bit-exact, squared distances within
1e-6 relative and in fact bit-identical).  Sizes span several build tiles
and finisher subtrees with ragged tails; the full 10M-point 3D workload is
checked by sampled queries against brute force and by properties that hold
at any size.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from bdl_inputs import (Op, clustered_points, random_op_sequence, uniform_points, workload)
from gpu_util import (assert_knn_equal, bits, compare_structure, log, run_parity, to_dev)

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


def _pair(bdl, d, leaf, X, idcap=1 << 22, knn_kernel=None, **kw):
    t = bdl.Tree(d, leaf_size=leaf, buffer_size=X, id_capacity=idcap, **kw)
    if knn_kernel is not None:
        t.set_param(bdl.PARAM_KNN_KERNEL, knn_kernel)
    return t, oracle.OracleBDL(d, leaf, X)


KERNELS = [0, 1, 3]  # one lane per query; one wavefront per 64 queries; one per query


def test_single_insert_small(torch, bdl):
    log("case: single insert d=2 n=100 X=16 leaf=4")
    t, o = _pair(bdl, 2, 4, 16)
    p = uniform_points(100, 2, 0)
    ids = np.arange(100, dtype=np.uint32)
    run_parity(t, o, [Op("insert", p, ids), Op("knn", uniform_points(50, 2, 1), k=3)], torch, 2,
               what="single")


@pytest.mark.parametrize("kern", KERNELS)
@pytest.mark.parametrize("X", [1024, 16])
def test_uniform2d_small_workload(torch, bdl, X, kern):
    """The 2D workload of 10x1000 inserts, 5x1000 erases and 1000 queries."""
    log(f"case: uniform2d_small X={X} kernel={kern}")
    w = workload("uniform2d_small", X=X)
    t, o = _pair(bdl, w.dim, w.leaf_size, X, knn_kernel=kern)
    run_parity(t, o, w.ops, torch, w.dim, what=f"uniform2d X={X}")


@pytest.mark.parametrize("seed,d,X,leaf,clustered", [
    (0, 2, 16, 4, False), (1, 3, 32, 16, False), (2, 5, 16, 2, True), (3, 1, 16, 16, False),
    (4, 7, 64, 16, True), (5, 16, 16, 8, False), (6, 3, 8, 1, True), (7, 9, 32, 5, False),
])
def test_random_ops(torch, bdl, seed, d, X, leaf, clustered):
    log(f"case: random ops seed={seed} d={d} X={X} leaf={leaf} clustered={clustered}")
    t, o = _pair(bdl, d, leaf, X)
    ops = list(random_op_sequence(seed, d, n_ops=40, max_batch=5 * X, id_capacity=1 << 22,
                                  clustered=clustered))
    run_parity(t, o, ops, torch, d, what=f"random seed={seed}")


@pytest.mark.parametrize("kern", KERNELS)
@pytest.mark.parametrize("d,n", [(3, 200_000), (2, 150_001), (7, 90_000), (16, 40_000)])
def test_large_levels_use_global_passes(torch, bdl, d, n, kern):
    """Trees larger than the LDS finisher go through the per-depth global
    passes (several 2048-point tiles per node) before the finisher."""
    log(f"case: large level d={d} n={n} kernel={kern}")
    t, o = _pair(bdl, d, 16, 1024, knn_kernel=kern)
    p = uniform_points(n, d, 10 + d)
    ids = (np.arange(n, dtype=np.uint32) * 7 + 3)
    ops = [Op("insert", p[: n // 3], ids[: n // 3]), Op("insert", p[n // 3:], ids[n // 3:]),
           Op("knn", uniform_points(3000, d, 20), k=8)]
    e = np.random.default_rng(d).choice(n, n // 3, replace=False)
    ops.append(Op("erase", p[e], ids[e]))
    ops.append(Op("knn", uniform_points(5000, d, 21), k=5))
    run_parity(t, o, ops, torch, d, what=f"large d={d}")


def test_unsorted_small_batches_both_kernels(torch, bdl):
    """Batches below the ordering threshold run in input order; a batch
    whose size is not a multiple of the wavefront leaves idle lanes."""
    log("case: small unsorted batches")
    d = 3
    for kern in KERNELS:
        t, o = _pair(bdl, d, 8, 32, knn_kernel=kern)
        p = uniform_points(3000, d, 40)
        ids = np.arange(3000, dtype=np.uint32)
        ops = [Op("insert", p, ids)]
        for nq in (1, 63, 65, 200, 4095, 4097):
            ops.append(Op("knn", uniform_points(nq, d, 41 + nq), k=6))
        run_parity(t, o, ops, torch, d, check_structure=False, what=f"small kern={kern}")


def test_coincident_points_larger_than_finisher(torch, bdl):
    """Thousands of identical points form one leaf that is copied out whole
    by the global pass (a node whose points all coincide is a leaf)."""
    log("case: coincident points")
    d = 3
    p = uniform_points(20000, d, 3)
    p[:6000] = p[0]
    p[6000:9000] = p[1]
    ids = np.arange(20000, dtype=np.uint32)
    t, o = _pair(bdl, d, 16, 1024)
    q = np.concatenate([p[:5], uniform_points(2000, d, 4)])
    run_parity(t, o, [Op("insert", p, ids), Op("knn", q, k=20),
                      Op("erase", p[:3000], ids[:3000]), Op("knn", q, k=7)], torch, d,
               what="coincident")


def test_deep_trees_and_depth_cap(torch, bdl):
    """A geometric sequence along one axis makes the spatial median peel off
    one point per split, so the tree reaches the depth cap (63) where an
    oversized leaf is allowed; tight clusters are mixed in."""
    log("case: deep trees")
    d = 3
    geo = np.full((400, d), 0.5, np.float32)
    geo[:, 0] = (2.0 ** (-np.arange(400) / 3.0)).astype(np.float32)
    p = np.concatenate([geo, clustered_points(30000, d, 5, n_clusters=4,
                                              log10_sigma=(-7.0, -6.0))]).astype(np.float32)
    ids = np.arange(len(p), dtype=np.uint32)
    t, o = _pair(bdl, d, 16, 1024)
    q = np.concatenate([p[::53], geo[::7] * np.float32(1.0001), uniform_points(500, d, 6)])
    run_parity(t, o, [Op("insert", p, ids), Op("knn", q.astype(np.float32), k=10)], torch, d,
               what="deep")
    info = o.level_info()
    heights = [int(o.export_level(j)[2]["depth"].max()) for j in bits(info["F"])]
    assert max(heights) == 63


@pytest.mark.parametrize("kern", KERNELS)
@pytest.mark.parametrize("k", [1, 2, 5, 10, 16, 17, 33, 64])
def test_knn_k_range(torch, bdl, k, kern):
    log(f"case: k={k} kernel={kern}")
    d = 3
    t, o = _pair(bdl, d, 16, 64, knn_kernel=kern)
    p = uniform_points(5000, d, 30)
    ids = np.arange(5000, dtype=np.uint32)
    run_parity(t, o, [Op("insert", p, ids), Op("knn", uniform_points(6000, d, 31), k=k)], torch,
               d, check_structure=False, what=f"k={k}")


def test_edge_cases(torch, bdl):
    log("case: edge cases")
    d = 2
    t, o = _pair(bdl, d, 4, 8, idcap=1000)
    q = uniform_points(10, d, 1)
    # empty tree: every row is padding
    gi, gd = t.knn(to_dev(q, torch), 4)
    t.sync()
    assert np.all(gi.cpu().numpy().view(np.uint32) == 0xFFFFFFFF)
    assert np.all(np.isinf(gd.cpu().numpy()))
    # n = 0 no-ops
    t.insert(torch.empty((0, d), dtype=torch.float32, device="cuda"),
             torch.empty(0, dtype=torch.int32, device="cuda"))
    assert t.erase(torch.empty((0, d), dtype=torch.float32, device="cuda"),
                   torch.empty(0, dtype=torch.int32, device="cuda")) == 0
    p = uniform_points(5, d, 2)
    ids = np.array([0, 5, 999, 3, 7], np.uint32)
    run_parity(t, o, [Op("insert", p, ids), Op("knn", q, k=9)], torch, d, what="edge")
    # erase: ids beyond capacity, wrong coordinates, repeats, never inserted
    ep = np.concatenate([p, p[:2], p[:1] + 1, p[:1]])
    eid = np.array([0, 5, 999, 3, 7, 0, 5, 0, 4000], np.uint32)
    assert t.erase(to_dev(ep, torch), to_dev(eid, torch)) == o.erase(ep, eid) == 5
    compare_structure(t, o, d, "edge after erase")
    with pytest.raises(bdl.BdlError):
        t.knn(to_dev(q, torch), 0)
    with pytest.raises(bdl.BdlError):
        t.knn(to_dev(q, torch), 65)
    t.close()


def test_check_inputs_rejects_bad_batches(torch, bdl):
    log("case: check_inputs")
    d = 2
    t = bdl.Tree(d, leaf_size=4, buffer_size=8, id_capacity=100, check_inputs=True)
    p = uniform_points(10, d, 0)
    t.insert(to_dev(p, torch), to_dev(np.arange(10, dtype=np.uint32), torch))
    for bad_p, bad_i in ((p, np.arange(90, 100, dtype=np.uint32) + 5),   # id >= capacity
                         (p, np.arange(10, dtype=np.uint32)),            # already live
                         (np.where(np.arange(20).reshape(10, 2) == 3, np.inf, p).astype(np.float32),
                          np.arange(20, 30, dtype=np.uint32))):          # not finite
        with pytest.raises(bdl.BdlError) as ei:
            t.insert(to_dev(bad_p, torch), to_dev(bad_i, torch))
        assert ei.value.code == bdl.BDL_EINVAL
    assert t.size() == 10
    t.close()


def test_drain_to_empty_with_half_rule(torch, bdl):
    """Erase 10% batches until empty (the paper's deletion experiment shape,
    scaled down): every half-capacity rebuild matches the oracle."""
    log("case: drain")
    d, X = 3, 64
    n = 20000
    t, o = _pair(bdl, d, 16, X)
    p = uniform_points(n, d, 8)
    ids = np.arange(n, dtype=np.uint32)
    ops = [Op("insert", p[i:i + 2000], ids[i:i + 2000]) for i in range(0, n, 2000)]
    order = np.random.default_rng(9).permutation(n)
    q = uniform_points(500, d, 9)
    for s in range(0, n, 2000):
        e = order[s:s + 2000]
        ops.append(Op("erase", p[e], ids[e]))
        ops.append(Op("knn", q, k=5))
    run_parity(t, o, ops, torch, d, what="drain")
    assert t.size() == 0 and t.level_info()["F"] == 0
    assert o.level_info()["reinserted"] > 0


@pytest.mark.parametrize("d,k,stack", [(3, 5, 130), (3, 64, 130), (16, 64, 130), (16, 17, 2048),
                                       (7, 10, 300)])
def test_query_wave_kernel_stack_limits(torch, bdl, d, k, stack):
    """One wavefront per query with a small pending-node stack: subtrees that
    do not fit are walked through parent links instead.  Clustered points
    with exact duplicates, several trees and a buffer."""
    log(f"case: query kernel d={d} k={k} stack={stack}")
    t, o = _pair(bdl, d, 8, 64, knn_kernel=3)
    t.set_param(bdl.PARAM_QUERY_STACK, stack)
    p = clustered_points(30_000, d, 50 + d, n_clusters=6)
    p[1000:1400] = p[5]
    ids = np.arange(30_000, dtype=np.uint32)
    q = np.concatenate([clustered_points(700, d, 60 + d, n_clusters=6), p[::97],
                        uniform_points(300, d, 61)]).astype(np.float32)
    ops = [Op("insert", p[:20_000], ids[:20_000]), Op("insert", p[20_000:], ids[20_000:]),
           Op("knn", q, k=k), Op("erase", p[::3], ids[::3]), Op("knn", q, k=k)]
    run_parity(t, o, ops, torch, d, check_structure=False, what=f"query d={d} k={k}")


def test_memory_budget_enomem_leaves_the_tree_unchanged(torch, bdl):
    """A tree with a device-memory budget: the insert that needs a new
    static tree beyond the budget fails with BDL_ENOMEM before anything is
    enqueued, the structure and the results stay those of the oracle that
    never saw that insert, and later operations within the budget work."""
    log("case: memory budget")
    d, X = 3, 256
    t = bdl.Tree(d, leaf_size=16, buffer_size=X, id_capacity=1 << 20, mem_budget=48 << 20)
    o = oracle.OracleBDL(d, 16, X)
    p = uniform_points(400_000, d, 70)
    ids = np.arange(400_000, dtype=np.uint32)
    done, failed = 0, False
    for s0 in range(0, 400_000, 20_000):
        try:
            t.insert(to_dev(p[s0:s0 + 20_000], torch), to_dev(ids[s0:s0 + 20_000], torch))
        except bdl.BdlError as e:
            assert e.code == bdl.BDL_ENOMEM
            failed = True
            break
        o.insert(p[s0:s0 + 20_000], ids[s0:s0 + 20_000])
        done = s0 + 20_000
    assert failed and done > 0
    compare_structure(t, o, d, "after ENOMEM")
    q = uniform_points(3000, d, 71)
    gi, gd = t.knn(to_dev(q, torch), 6)
    t.sync()
    oi, od = o.knn(q, 6)
    assert_knn_equal(gi.cpu().numpy(), gd.cpu().numpy(), oi, od, "knn after ENOMEM")
    # the tree keeps working: an erase either fails before changing anything
    # or takes effect; a small insert fits in the arenas already held
    e = ids[:done:7]
    try:
        ne = t.erase(to_dev(p[e.astype(np.int64)], torch), to_dev(e, torch))
        assert ne == o.erase(p[e.astype(np.int64)], e)
    except bdl.BdlError as err:
        assert err.code == bdl.BDL_ENOMEM
    compare_structure(t, o, d, "after erase")
    t.insert(to_dev(p[done:done + 100], torch), to_dev(ids[done:done + 100], torch))
    o.insert(p[done:done + 100], ids[done:done + 100])
    compare_structure(t, o, d, "after recovery")
    gi, gd = t.knn(to_dev(q, torch), 6)
    t.sync()
    oi, od = o.knn(q, 6)
    assert_knn_equal(gi.cpu().numpy(), gd.cpu().numpy(), oi, od, "knn after recovery")
    t.close()
