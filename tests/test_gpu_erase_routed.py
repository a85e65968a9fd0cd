"""Erase_S with Bloom prefilters (Alg. 2, Section V-A) against the oracle.

With BDL_PARAM_ERASE_ROUTE = 1 bdl_erase finds each (point, id) pair by
testing every tree's Bloom filter and descending the trees that may hold it
along their splits, instead of through the id map.  The results must be the
same: erased counts, the trees (slots, points, nodes bit for bit), the live
counts and every k-NN row equal the oracle's, whose erase routes points the
same way.  The cases cover filters built lazily after rebuilds, points in
the buffer, coordinates that equal split values, repeated ids, wrong
coordinates and never-inserted ids, both split rules and both baselines.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from bdl_inputs import Op, clustered_points, random_op_sequence, uniform_points
from gpu_util import compare_structure, log, run_parity, to_dev

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


def _routed(bdl, d, leaf, X, split="spatial", structure="bdl", idcap=1 << 22):
    t = bdl.Tree(d, leaf_size=leaf, buffer_size=X, id_capacity=idcap, split=split,
                 structure=structure)
    t.set_param(bdl.PARAM_ERASE_ROUTE, 1)
    return t, oracle.OracleBDL(d, leaf, X, split=split, mode=structure)


@pytest.mark.parametrize("seed,d,leaf,X,clustered,split", [
    (0, 2, 4, 64, False, "spatial"), (1, 3, 16, 128, True, "spatial"),
    (2, 7, 8, 32, True, "object"), (3, 1, 2, 16, False, "spatial"),
    (4, 16, 16, 64, False, "object"), (5, 5, 1, 8, True, "spatial"),
])
def test_routed_erase_random_ops(torch, bdl, seed, d, leaf, X, clustered, split):
    log(f"case: routed erase random ops seed={seed} d={d} leaf={leaf} X={X} {split}")
    t, o = _routed(bdl, d, leaf, X, split=split)
    ops = list(random_op_sequence(100 + seed, d, n_ops=40, max_batch=500,
                                  id_capacity=1 << 22, clustered=clustered))
    run_parity(t, o, ops, torch, d, what=f"routed seed={seed}")
    t.close()


@pytest.mark.parametrize("structure", ["rebuild_all", "no_rebuild"])
def test_routed_erase_baselines(torch, bdl, structure):
    """B2's leaves grow past the leaf size and keep tombstones; B1 rebuilds
    after each erase that hits (its filter is rebuilt lazily)."""
    log(f"case: routed erase {structure}")
    d = 3
    t, o = _routed(bdl, d, 16, 64, structure=structure)
    base = uniform_points(40_000, d, 300)
    hot = clustered_points(20_000, d, 301, n_clusters=1, log10_sigma=(-2.5, -2.5))
    ids = np.arange(60_000, dtype=np.uint32)
    q = np.concatenate([hot[::40], uniform_points(500, d, 302)]).astype(np.float32)
    ops = [Op("insert", base, ids[:40_000]), Op("erase", base[::5], ids[:40_000:5]),
           Op("insert", hot[:10_000], ids[40_000:50_000]), Op("knn", q, k=5),
           Op("erase", hot[:10_000:3], ids[40_000:50_000:3]),
           Op("erase", base[1::5], ids[1:40_000:5]),
           Op("insert", hot[10_000:], ids[50_000:]), Op("knn", q, k=8),
           Op("erase", np.concatenate([hot[10_000::2], base[::5]]),
              np.concatenate([ids[50_000::2], ids[:40_000:5]])), Op("knn", q, k=5)]
    run_parity(t, o, ops, torch, d, what=f"routed {structure}")
    t.close()


def test_routed_erase_on_split_values(torch, bdl):
    """Integer grid points: many coordinates equal a split value, so routing
    must send x == split to the right child exactly as the build did."""
    log("case: routed erase grid")
    d = 2
    g = np.stack(np.meshgrid(np.arange(64), np.arange(64), indexing="ij"), -1)
    pts = np.concatenate([g.reshape(-1, d)] * 3).astype(np.float32)  # each point 3 times
    rng = np.random.default_rng(7)
    perm = rng.permutation(len(pts))
    pts = pts[perm]
    ids = np.arange(len(pts), dtype=np.uint32)
    t, o = _routed(bdl, d, 4, 32)
    ops = []
    for s in range(0, len(pts), 1500):
        ops.append(Op("insert", pts[s:s + 1500], ids[s:s + 1500]))
        e = rng.choice(s + min(1500, len(pts) - s), size=300, replace=False)
        ops.append(Op("erase", pts[e], ids[e]))
    ops.append(Op("knn", uniform_points(300, d, 8) * 64, k=6))
    run_parity(t, o, ops, torch, d, what="grid")
    t.close()


def test_routed_equals_map_erase_large(torch, bdl):
    """600k clustered 3D points in 10 batches with erases between them: the
    routed erase and the id-map erase leave identical trees (and both equal
    the oracle's)."""
    log("case: routed vs map erase 600k")
    d, n, b = 3, 600_000, 60_000
    pts = clustered_points(n, d, 310, log10_sigma=(-4.0, -1.0))
    ids = np.arange(n, dtype=np.uint32)
    rng = np.random.default_rng(311)
    dp, di = to_dev(pts, torch), to_dev(ids, torch)
    tr, o = _routed(bdl, d, 16, 1024, idcap=n)
    tm = bdl.Tree(d, leaf_size=16, buffer_size=1024, id_capacity=n)
    alive = np.zeros(n, bool)
    for s in range(0, n, b):
        for t in (tr, tm):
            t.insert(dp[s:s + b], di[s:s + b])
        o.insert(pts[s:s + b], ids[s:s + b])
        alive[s:s + b] = True
        live = np.flatnonzero(alive)
        e = rng.choice(live, size=len(live) // 10, replace=False)
        # a few wrong coordinates and never-inserted ids ride along
        ep = pts[e].copy()
        ep[::97, 0] += np.float32(1e-3)
        ei = ids[e].copy()
        ei[1::89] = np.uint32(n + 5)
        dep, dei = to_dev(ep, torch), to_dev(ei, torch)
        er = tr.erase(dep, dei)
        em = tm.erase(dep, dei)
        eo = o.erase(ep, ei)
        assert er == em == eo, f"batch {s // b}: routed {er} map {em} oracle {eo}"
        ok = np.ones(len(e), bool)
        ok[::97] = False
        ok[1::89] = False
        alive[e[ok]] = False
    compare_structure(tr, o, d, "routed 600k")
    compare_structure(tm, o, d, "map 600k")
    tr.close()
    tm.close()
