"""Parity of the object-median build (Section V-C) with the CPU oracle.

With BDL_FLAG_OBJECT_MEDIAN every tree splits a node at its coordinate of
rank floor(count/2) in the split dimension.  The GPU finds it by a radix
select over the ordered keys of the coordinates (four 8-bit rounds per
depth of the global passes, eight 4-bit rounds in the LDS finisher); the
oracle sorts them.  After every operation the static trees (slot order,
points, node arrays in vEB order, split values bit for bit), the buffer and
the live counts are compared, and every k-NN row.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from bdl_inputs import Op, clustered_points, random_op_sequence, uniform_points
from gpu_util import bits, log, run_parity

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


def _pair(bdl, d, leaf, X, idcap=1 << 22):
    t = bdl.Tree(d, leaf_size=leaf, buffer_size=X, id_capacity=idcap, split="object")
    return t, oracle.OracleBDL(d, leaf, X, split="object")


@pytest.mark.parametrize("seed,d,X,leaf,clustered", [
    (0, 2, 16, 4, False), (1, 3, 32, 16, False), (2, 5, 16, 2, True), (3, 1, 16, 16, False),
    (4, 7, 64, 16, True), (5, 16, 16, 8, False), (6, 3, 8, 1, True),
])
def test_object_median_random_ops(torch, bdl, seed, d, X, leaf, clustered):
    log(f"case: object median random ops seed={seed} d={d} X={X} leaf={leaf}")
    t, o = _pair(bdl, d, leaf, X)
    ops = list(random_op_sequence(seed, d, n_ops=30, max_batch=5 * X, id_capacity=1 << 22,
                                  clustered=clustered))
    run_parity(t, o, ops, torch, d, what=f"object random seed={seed}")
    t.close()


@pytest.mark.parametrize("d,n,clustered", [(3, 200_000, False), (2, 150_001, True),
                                           (7, 90_000, True), (16, 40_000, False)])
def test_object_median_global_passes(torch, bdl, d, n, clustered):
    """Trees above the finisher threshold select their medians in the global
    passes (many tiles per node, ragged tails), then in the LDS finisher."""
    log(f"case: object median large d={d} n={n} clustered={clustered}")
    t, o = _pair(bdl, d, 16, 1024)
    p = clustered_points(n, d, 80 + d, n_clusters=7) if clustered else uniform_points(n, d, 80 + d)
    ids = np.arange(n, dtype=np.uint32) * 5 + 1
    e = np.random.default_rng(d).choice(n, n // 4, replace=False)
    ops = [Op("insert", p[: n // 3], ids[: n // 3]), Op("insert", p[n // 3:], ids[n // 3:]),
           Op("knn", uniform_points(3000, d, 81), k=8), Op("erase", p[e], ids[e]),
           Op("knn", np.concatenate([p[::101], uniform_points(2000, d, 82)]), k=5)]
    run_parity(t, o, ops, torch, d, what=f"object large d={d}")
    # the object median halves: no tree is deeper than repeated halving allows
    # beyond the coincident-point leaves
    info = o.level_info()
    for j in bits(info["F"]):
        ids_j, _, nodes = o.export_level(j)
        m, h = len(ids_j), 1
        while m > 16:
            m -= m // 2
            h += 1
        assert int(nodes["depth"].max()) + 1 <= h + 2
    t.close()


def test_object_median_duplicates(torch, bdl):
    """Many equal coordinates: medians at the minimum (split at the maximum),
    coincident points beyond the finisher size, repeated median values."""
    log("case: object median duplicates")
    d = 3
    p = uniform_points(30_000, d, 90)
    p[:7000, 0] = p[0, 0]          # a third of the points share one x
    p[7000:12_000] = p[1]          # 5000 coincident points
    p[12_000:20_000, 1] = np.float32(0.25)
    p[20_000:20_050] = -0.0        # signed zeros
    p[20_050:20_100] = 0.0
    ids = np.arange(30_000, dtype=np.uint32)
    t, o = _pair(bdl, d, 8, 512)
    q = np.concatenate([p[::97], uniform_points(1000, d, 91)]).astype(np.float32)
    run_parity(t, o, [Op("insert", p[:16_000], ids[:16_000]),
                      Op("insert", p[16_000:], ids[16_000:]), Op("knn", q, k=12),
                      Op("erase", p[::5], ids[::5]), Op("knn", q, k=4)], torch, d,
               what="object duplicates")
    t.close()
