"""bdl_knn_noalloc: the k-NN entry point that allocates no device memory.

Its results must equal bdl_knn's on the same tree and queries (ids bit for
bit, squared distances bit-identical and so within 1e-6 relative), on two
calls in a row where the second is smaller, so that the second call reuses
the device's static scratch after the first left its contents there.  Both
large calls take the Hilbert-ordered path that uses the scratch; a small
call takes the wavefront-per-query path that uses none.  Rows are also
checked against the oracle's brute force.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from bdl_inputs import uniform_points
from gpu_util import assert_knn_equal, log, to_dev

pytestmark = pytest.mark.gpu

MAX_Q = 1 << 20


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


def _both(tree, q, k):
    a_i, a_d = tree.knn(q, k)
    b_i, b_d = tree.knn_noalloc(q, k)
    tree.sync()
    return (a_i.cpu().numpy(), a_d.cpu().numpy(), b_i.cpu().numpy(), b_d.cpu().numpy())


def test_noalloc_equals_knn_on_two_calls(torch, bdl):
    d, n = 3, 400_000
    log(f"case: noalloc d={d} n={n}: build")
    pts = uniform_points(n, d, 31)
    ids = np.arange(n, dtype=np.uint32)
    t = bdl.Tree(d, leaf_size=16, buffer_size=1024, id_capacity=1 << 20)
    for s in range(0, n, 100_000):
        t.insert(to_dev(pts[s:s + 100_000], torch), to_dev(ids[s:s + 100_000], torch))
    # first call: dense queries, wavefront-per-group kernel on a persistent
    # grid with Hilbert ordering; second call smaller, lane kernel, ordered
    for nq, k, kern, seed in ((700_000, 5, bdl.KNN_WAVE, 32), (150_000, 10, bdl.KNN_LANE, 33)):
        log(f"case: noalloc nq={nq} k={k} kernel={kern}")
        t.set_param(bdl.PARAM_KNN_KERNEL, kern)
        q = to_dev(uniform_points(nq, d, seed), torch)
        a_i, a_d, b_i, b_d = _both(t, q, k)
        assert_knn_equal(b_i, b_d, a_i.view(np.uint32), a_d, f"noalloc vs knn nq={nq}")
        rows = np.random.default_rng(seed).choice(nq, 48, replace=False)
        oi, od = oracle.bruteforce_knn(pts, ids, q.cpu().numpy()[rows], k)
        assert_knn_equal(b_i[rows], b_d[rows], oi, od, f"noalloc vs brute force nq={nq}")
    log("case: noalloc small batch (no ordering)")
    t.set_param(bdl.PARAM_KNN_KERNEL, bdl.KNN_AUTO)
    q = to_dev(uniform_points(1000, d, 34), torch)
    a_i, a_d, b_i, b_d = _both(t, q, 5)
    assert_knn_equal(b_i, b_d, a_i.view(np.uint32), a_d, "noalloc small")
    t.close()


def test_noalloc_rejects_batches_beyond_its_scratch(torch, bdl):
    log("case: noalloc size limit")
    t = bdl.Tree(2, leaf_size=16, buffer_size=64, id_capacity=1 << 12)
    p = uniform_points(500, 2, 35)
    t.insert(to_dev(p, torch), to_dev(np.arange(500, dtype=np.uint32), torch))
    q = torch.zeros((MAX_Q + 1, 2), dtype=torch.float32, device="cuda")
    with pytest.raises(bdl.BdlError) as e:
        t.knn_noalloc(q, 3)
    assert e.value.code == bdl.BDL_EINVAL
    # the largest allowed batch runs and equals bdl_knn
    q = to_dev(uniform_points(MAX_Q, 2, 36), torch)
    t.set_param(bdl.PARAM_KNN_KERNEL, bdl.KNN_LANE)
    a_i, a_d, b_i, b_d = _both(t, q, 3)
    assert_knn_equal(b_i, b_d, a_i.view(np.uint32), a_d, "noalloc at capacity")
    t.close()
