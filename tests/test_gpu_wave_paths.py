"""The wavefront-per-group kNN_L kernel on the paths that only large batches
and particular trees take.

For d <= 3 and k <= 5 a batch of at least 2M queries runs with two queries
per lane (128 per wavefront); smaller batches with one.  In a forest whose
trees are all balanced the near child of a split is entered without a prune
test; clustered points give deep trees, where it is tested.  Whatever the
path, every query's row is the exact kNN_L row: one launch of 2M + 12345
queries (two per lane) must equal, bit for bit, the same queries in two
launches of under 2M (one per lane), and sampled rows must equal the
brute-force definition over the live points.  Uniform 3D points give
balanced trees, clustered 2D points skewed ones.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from bdl_inputs import clustered_points, uniform_points
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


@pytest.mark.parametrize("name,d,clustered,k", [
    ("uniform3d", 3, False, 5), ("uniform3d", 3, False, 2),
    ("clustered2d", 2, True, 5), ("uniform1d", 1, False, 4),
])
def test_two_queries_per_lane_equal_one(torch, bdl, name, d, clustered, k):
    log(f"case: group kernel paths {name} k={k}")
    n = 600_000
    pts = clustered_points(n, d, 60) if clustered else uniform_points(n, d, 60)
    ids = np.arange(n, dtype=np.uint32)
    t = bdl.Tree(d, leaf_size=16, buffer_size=1024, id_capacity=n)
    t.set_param(bdl.PARAM_KNN_KERNEL, 1)
    dp, di = to_dev(pts, torch), to_dev(ids, torch)
    for s in range(0, n, n // 6):
        t.insert(dp[s:s + n // 6], di[s:s + n // 6])
    e = np.sort(np.random.default_rng(61).choice(n, n // 10, replace=False))
    ed = torch.from_numpy(e).cuda()
    assert t.erase(dp[ed], di[ed]) == len(e)
    live = np.ones(n, bool)
    live[e] = False
    # queries: live and erased points with a small jitter, and points drawn
    # over the set's bounding box; a count that is no multiple of 128
    rng = np.random.default_rng(62)
    nq = (1 << 21) + 12_345
    near = pts[rng.integers(0, n, nq // 2)] + rng.normal(0, 1e-4, (nq // 2, d)).astype(np.float32)
    lo, hi = pts.min(0), pts.max(0)
    far = (lo + (hi - lo) * rng.random((nq - nq // 2, d))).astype(np.float32)
    q = np.concatenate([near, far]).astype(np.float32)
    q = q[rng.permutation(nq)]
    qd = to_dev(q, torch)
    one_i, one_d = t.knn(qd, k)
    h = nq // 2
    ai, ad = t.knn(qd[:h], k)
    bi, bd = t.knn(qd[h:], k)
    t.sync()
    assert torch.equal(one_i, torch.cat([ai, bi])), f"{name}: ids differ between the two paths"
    assert torch.equal(one_d.view(torch.int32), torch.cat([ad, bd]).view(torch.int32)), \
        f"{name}: distances differ between the two paths"
    sel = np.sort(rng.choice(nq, 64, replace=False))
    oi, od = oracle.bruteforce_knn(pts[live], ids[live], q[sel], k)
    assert_knn_equal(one_i.cpu().numpy()[sel], one_d.cpu().numpy()[sel], oi, od,
                     f"{name} sampled rows")
    t.close()
