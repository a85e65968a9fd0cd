"""Launch shapes of kNN_L: persistent grids with per-XCD work counters, the
shape table and the autotuner.  Every shape must give the same results bit
for bit, and the oracle's (checked on sampled rows against brute force)."""
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
    assert t.cuda.is_available()
    t.cuda.set_device(0)
    return t


@pytest.fixture(scope="module")
def bdl():
    import paper_2112_06188_amd as m
    m.load_library()
    return m


@pytest.fixture(scope="module")
def loaded(torch, bdl):
    """A 3D clustered tree of 300k points (several levels and a buffer) and
    1.5M queries: more groups of 64 than the device holds at once, so a
    persistent launch really draws from the work counters."""
    d = 3
    n = 300_000
    p = clustered_points(n, d, 11)
    ids = np.arange(n, dtype=np.uint32)
    t = bdl.Tree(d, leaf_size=16, buffer_size=1024, id_capacity=1 << 20)
    for i in range(0, n, 70_000):
        t.insert(to_dev(p[i:i + 70_000], torch), to_dev(ids[i:i + 70_000], torch))
    q = np.concatenate([clustered_points(1_000_000, d, 12), uniform_points(500_000, d, 13)])
    yield t, p, ids, q
    t.close()


def _check_sample(p, ids, q, gi, gd, k, what):
    rng = np.random.default_rng(3)
    sel = np.sort(rng.choice(len(q), size=300, replace=False))
    oi, od = oracle.bruteforce_knn(p, ids, q[sel], k)
    assert_knn_equal(gi.cpu().numpy()[sel], gd.cpu().numpy()[sel], oi, od, what)


@pytest.mark.parametrize("k", [5, 10, 24])
def test_persistent_grid_matches_plain_launch(torch, bdl, loaded, k):
    t, p, ids, q = loaded
    qd = to_dev(q, torch)
    base = None
    for kern in (1, 0):
        for block in (256, 64):
            for pers in (0, 1):
                log(f"case: k={k} kernel={kern} block={block} persistent={pers}")
                t.set_param(bdl.PARAM_KNN_KERNEL, kern)
                t.set_param(bdl.PARAM_KNN_BLOCK, block)
                t.set_param(bdl.PARAM_PERSISTENT, pers)
                gi, gd = t.knn(qd, k)
                t.sync()
                if base is None:
                    base = (gi, gd)
                    _check_sample(p, ids, q, gi, gd, k, f"k={k}")
                else:
                    assert torch.equal(gi, base[0])
                    assert torch.equal(gd.view(torch.int32), base[1].view(torch.int32))
    t.set_param(bdl.PARAM_KNN_KERNEL, bdl.KNN_AUTO)
    t.set_param(bdl.PARAM_KNN_BLOCK, 256)
    t.set_param(bdl.PARAM_PERSISTENT, 2)


def test_batched_persistent_with_graph_replays(torch, bdl, loaded):
    """bdl_knn_batch over more queries than the device holds, on a persistent
    grid, replayed from its graph three times."""
    t, p, ids, q = loaded
    t.set_param(bdl.PARAM_PERSISTENT, 1)
    cuts = [0, 1, 70_000, 300_001, 900_000, 1_500_000]
    ks = [5, 1, 10, 5, 2]
    qd = to_dev(q, torch)
    ref = [t.knn(qd[a:b], k) for a, b, k in zip(cuts, cuts[1:], ks)]
    for rep in range(3):
        log(f"case: batched persistent replay {rep}")
        outs = t.knn_batch([(qd[a:b], k) for a, b, k in zip(cuts, cuts[1:], ks)])
        t.sync()
        for (ri, rd), (gi, gd) in zip(ref, outs):
            assert torch.equal(gi, ri) and torch.equal(gd.view(torch.int32), rd.view(torch.int32))
    t.set_param(bdl.PARAM_PERSISTENT, 2)


def test_shape_table_routes_by_k_and_count(torch, bdl, loaded):
    t, p, ids, q = loaded
    rows = [dict(k_lo=1, k_hi=4, nq_lo=0, nq_hi=5000, kernel=0, block=64, persistent=0, sort=0),
            dict(k_lo=1, k_hi=64, nq_lo=0, nq_hi=1 << 40, kernel=1, block=128, persistent=1,
                 sort=1)]
    t.set_knn_shapes(rows)
    qd = to_dev(q, torch)
    for n, k in ((3000, 3), (3000, 7), (400_000, 3)):
        log(f"case: shape table n={n} k={k}")
        gi, gd = t.knn(qd[:n], k)
        t.sync()
        oi, od = oracle.bruteforce_knn(p, ids, q[:200], k)
        assert_knn_equal(gi.cpu().numpy()[:200], gd.cpu().numpy()[:200], oi, od, f"n={n} k={k}")
    with pytest.raises(bdl.BdlError):
        t.set_knn_shapes([dict(rows[0], block=96)])
    t.set_knn_shapes([])


def test_autotune_installs_a_table_that_keeps_results(torch, bdl):
    from paper_2112_06188_amd import autotune
    d = 4
    p = uniform_points(60_000, d, 21)
    ids = np.arange(60_000, dtype=np.uint32)
    t = bdl.Tree(d, leaf_size=16, buffer_size=256, id_capacity=1 << 17)
    t.insert(to_dev(p, torch), to_dev(ids, torch))
    qs = uniform_points(20_000, d, 22)
    qd = to_dev(qs, torch)
    log("case: autotune")
    res = autotune.tune(t, lambda n: qd[:n], k_bands=((1, 5), (6, 12)),
                        nq_bands=((1, 2000), (2001, 1 << 30)), max_nq=20_000, reps=1,
                        cands=autotune.candidates(blocks=(64, 256)))
    assert len(res["rows"]) == 4
    assert len(res["timings"]) == 4 * len(autotune.candidates(blocks=(64, 256)))
    for n, k in ((1500, 5), (20_000, 12)):
        gi, gd = t.knn(qd[:n], k)
        t.sync()
        oi, od = oracle.bruteforce_knn(p, ids, qs[:300], k)
        assert_knn_equal(gi.cpu().numpy()[:300], gd.cpu().numpy()[:300], oi, od, f"tuned k={k}")
    t.close()
