"""Parity of the baselines of Section III-B with the CPU oracle on the GPU.

B1 rebuilds its one kd-tree after every insert and every erase that removes
a point; B2 builds its tree from the first batch and afterwards inserts into
the existing leaves along the existing splits (boxes grow), leaving erased
points as tombstones.  After every operation the tree (slot order, points,
node arrays with their boxes and splits, bit for bit) and the live counts
are compared with the oracle's baseline of the same kind, and every k-NN row.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from bdl_inputs import Op, clustered_points, random_op_sequence, uniform_points
from gpu_util import log, run_parity

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


def _pair(bdl, mode, d, leaf, X=64, idcap=1 << 22, knn_kernel=None):
    t = bdl.Tree(d, leaf_size=leaf, buffer_size=X, id_capacity=idcap, structure=mode)
    if knn_kernel is not None:
        t.set_param(bdl.PARAM_KNN_KERNEL, knn_kernel)
    return t, oracle.OracleBDL(d, leaf, X, mode=mode)


MODES = ["rebuild_all", "no_rebuild"]


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("seed,d,leaf,clustered", [
    (0, 2, 4, False), (1, 3, 16, True), (2, 7, 8, True), (3, 1, 2, False), (4, 16, 16, False),
])
def test_baseline_random_ops(torch, bdl, mode, seed, d, leaf, clustered):
    log(f"case: baseline {mode} random ops seed={seed} d={d} leaf={leaf}")
    t, o = _pair(bdl, mode, d, leaf)
    ops = list(random_op_sequence(seed, d, n_ops=30, max_batch=400, id_capacity=1 << 22,
                                  clustered=clustered))
    run_parity(t, o, ops, torch, d, what=f"{mode} seed={seed}")
    t.close()


@pytest.mark.parametrize("kern", [0, 1, 3])
@pytest.mark.parametrize("mode", MODES)
def test_baseline_large_and_skewed(torch, bdl, mode, kern):
    """A tree above the finisher size, then batches concentrated in one
    cluster: B1 rebuilds every time, B2's leaves in that cluster grow far
    beyond the leaf size (its weakness), and erases hit both."""
    log(f"case: baseline {mode} large kernel={kern}")
    d = 3
    t, o = _pair(bdl, mode, d, 16, knn_kernel=kern)
    base = uniform_points(120_000, d, 90)
    hot = clustered_points(60_000, d, 91, n_clusters=1, log10_sigma=(-2.5, -2.5))
    ids = np.arange(180_000, dtype=np.uint32)
    q = np.concatenate([hot[::50], uniform_points(2000, d, 92)]).astype(np.float32)
    ops = [Op("insert", base, ids[:120_000]), Op("knn", q, k=5),
           Op("insert", hot[:30_000], ids[120_000:150_000]), Op("knn", q, k=5),
           Op("erase", base[::4], ids[:120_000:4]),
           Op("insert", hot[30_000:], ids[150_000:]), Op("knn", q, k=10),
           Op("erase", hot[::3], ids[120_000::3]), Op("knn", q, k=5)]
    run_parity(t, o, ops, torch, d, what=f"{mode} large")
    if mode == "no_rebuild":
        ids0, _, nodes = o.export_level(0)
        assert nodes["count"][nodes["dim"] < 0].max() > 16 * 20
    t.close()


def test_baselines_reject_both_flags(bdl):
    import ctypes
    L = bdl.load_library()
    h = ctypes.c_void_p()
    cfg = bdl.Config(3, 16, 64, 100, 0, bdl.FLAG_REBUILD_ALL | bdl.FLAG_NO_REBUILD)
    assert L.bdl_create(ctypes.byref(cfg), None, ctypes.byref(h)) == bdl.BDL_EINVAL
