"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these expectations comes from the oracle itself: they are the
paper's worked examples (tests/golden, each citing its passage), closed forms
of the logarithmic method, exact arithmetic on inputs where float32 is exact,
a library kd-tree in float64 with the float32 error bound, and structural
invariants checked by tests/treecheck.py.
"""
from __future__ import annotations

import json
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from bdl_inputs import clustered_points, random_op_sequence, uniform_points
from treecheck import check_tree, veb_key

GOLD = os.path.join(os.path.dirname(__file__), "golden")
U = 2.0 ** -24


def _gold(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


# --------------------------------------------------------------------------
# result definition
# --------------------------------------------------------------------------

@pytest.mark.parametrize("d,k", [(1, 1), (2, 5), (3, 5), (5, 10), (7, 10), (16, 3)])
def test_bruteforce_matches_scipy_kdtree_within_fp32_bound(d, k):
    """The brute-force definition against scipy's kd-tree in float64: the
    float32 squared distances lie within (d+3) u of the exact ones, and
    wherever the k-th and (k+1)-th exact distances are separated by more
    than that bound, the id sets agree."""
    from scipy.spatial import cKDTree

    rng = np.random.default_rng(100 + d)
    n = 3000
    pts = rng.random((n, d), dtype=np.float32)
    ids = rng.permutation(n).astype(np.uint32) + np.uint32(7)
    q = rng.random((300, d), dtype=np.float32)
    oi, od = oracle.bruteforce_knn(pts, ids, q, k)
    tree = cKDTree(pts.astype(np.float64))
    _, nb = tree.query(q.astype(np.float64), k=k + 1)
    nb = nb.reshape(len(q), k + 1)
    tol = (d + 3) * U
    id2row = {int(v): i for i, v in enumerate(ids)}
    checked = 0
    for r in range(len(q)):
        rows = np.array([id2row[int(v)] for v in oi[r]])
        exact = ((pts[rows].astype(np.float64) - q[r].astype(np.float64)) ** 2).sum(axis=1)
        assert np.all(np.abs(od[r].astype(np.float64) - exact) <= tol * exact + 1e-45)
        ex_nb = ((pts[nb[r]].astype(np.float64) - q[r].astype(np.float64)) ** 2).sum(axis=1)
        if ex_nb[k] - ex_nb[k - 1] > 3 * tol * ex_nb[k]:
            assert set(int(v) for v in oi[r]) == set(int(ids[j]) for j in nb[r][:k])
            checked += 1
        assert np.all(np.diff(od[r]) >= 0)
    assert checked > 250


def _exact_knn(pts, ids, q, k):
    """Exact rational k-NN with (d2, id) order; padding (TOMB, inf)."""
    out_i = np.full((len(q), k), oracle.TOMB, np.uint32)
    out_d = np.full((len(q), k), np.inf, np.float64)
    for r, qq in enumerate(q):
        keys = []
        for p, i in zip(pts, ids):
            s = sum((Fraction(float(a)) - Fraction(float(b))) ** 2 for a, b in zip(qq, p))
            keys.append((s, int(i)))
        keys.sort()
        for j, (s, i) in enumerate(keys[:k]):
            out_i[r, j] = i
            out_d[r, j] = float(s)
    return out_i, out_d


@pytest.mark.parametrize("d", [1, 2, 3])
def test_lattice_ties_exact(d):
    """Integer lattice with duplicated points: float32 is exact here, so the
    exact rational answer (ties broken by the smaller id, short rows padded)
    is the expected value bit for bit."""
    rng = np.random.default_rng(5 + d)
    n = 150
    pts = rng.integers(0, 5, size=(n, d)).astype(np.float32)
    pts[:20] = pts[20:40]  # exact duplicates
    ids = rng.permutation(1000)[:n].astype(np.uint32)
    q = (rng.integers(0, 9, size=(40, d)) / 2.0).astype(np.float32)
    for k in (1, 4, 9):
        ei, ed = _exact_knn(pts, ids, q, k)
        oi, od = oracle.bruteforce_knn(pts, ids, q, k)
        assert np.array_equal(oi, ei)
        assert np.array_equal(od.astype(np.float64), ed)
    # fewer live points than k: padding
    ei, ed = _exact_knn(pts[:3], ids[:3], q, 6)
    oi, od = oracle.bruteforce_knn(pts[:3], ids[:3], q, 6)
    assert np.array_equal(oi, ei) and np.array_equal(od.astype(np.float64), ed)
    assert np.all(oi[:, 3:] == oracle.TOMB) and np.all(np.isinf(od[:, 3:]))


def test_dist2_canonical_negative_zero_and_self():
    a = np.array([0.25, -0.0, 3.0], np.float32)
    b = np.array([0.25, 0.0, 3.0], np.float32)
    assert oracle.dist2(a, b) == 0.0
    assert oracle.dist2(a, a) == 0.0


# --------------------------------------------------------------------------
# static tree: BuildvEB with the spatial median
# --------------------------------------------------------------------------

def test_veb_layout_fig3_example():
    g = _gold("veb_fig3.json")
    pts = np.array(g["points"], np.float32)
    p, i, nodes, h = oracle.tree_build(pts, np.arange(len(pts)), g["leaf_size"])
    assert h == g["levels"]
    assert len(nodes) == 2 ** g["levels"] - 1
    for idx in g["top_indices"]:
        assert nodes[idx]["depth"] < 2
    assert [int(nodes[j]["depth"]) for j in g["top_indices"]] == [0, 1, 1]
    # bottom subtree roots: depth 2, left to right, at the cited offsets,
    # each followed by its own two children
    for j, s in enumerate(g["bottom_subtree_starts"]):
        assert nodes[s]["depth"] == 2 and int(nodes[s]["path"]) == j
        kids = {int(nodes[s]["left"]), int(nodes[s]["right"])}
        assert kids == {s + 1, s + 2}
    assert nodes[1]["path"] == 0 and nodes[2]["path"] == 1
    check_tree(p, i, nodes, g["leaf_size"])


def test_veb_key_matches_fig3_offsets():
    # the independent key formula reproduces the same worked example
    assert [veb_key(4, 0, 0), veb_key(4, 1, 0), veb_key(4, 1, 1)] == [0, 1, 2]
    assert [veb_key(4, 2, j) for j in range(4)] == [3, 6, 9, 12]


def test_spatial_median_fig1():
    g = _gold("fig1_split.json")
    for part in ("before", "after"):
        pts = np.array(g[part]["points"], np.float32)
        p, i, nodes, h = oracle.tree_build(pts, np.arange(len(pts)), g["leaf_size"])
        assert nodes[0]["dim"] == g[part]["root_dim"]
        assert np.float32(nodes[0]["split"]) == np.float32(g[part]["root_split"])
        check_tree(p, i, nodes, g["leaf_size"])


def _node_at(nodes, path):
    """Node reached from the root by a string of L/R moves."""
    i = 0
    for m in path:
        assert nodes[i]["dim"] >= 0, f"path {path!r} runs into a leaf"
        i = int(nodes[i]["left"] if m == "L" else nodes[i]["right"])
    return i


def _slot_points(p, nodes, i):
    nd = nodes[i]
    rows = p[int(nd["begin"]):int(nd["begin"]) + int(nd["count"])]
    return sorted(tuple(float(v) for v in r) for r in rows)


_SPATIAL_CASES = _gold("spatial_median.json")["cases"]


@pytest.mark.parametrize("case", _SPATIAL_CASES, ids=[c["name"] for c in _SPATIAL_CASES])
def test_spatial_median_split_values(case):
    """Hand-derived split values and sides (Section V-C) where the midpoint
    of the tight extent differs from the mean and the object median, plus the
    zero-extent dimension skip and the two fix-ups that keep both sides
    non-empty (adjacent floats, overflowing sum)."""
    pts = np.array(case["points"], np.float32)
    p, i, nodes, h = oracle.tree_build(pts, np.arange(len(pts)), case["leaf_size"])
    for want in case["nodes"]:
        n = _node_at(nodes, want["path"])
        nd = nodes[n]
        assert int(nd["dim"]) == want["dim"], want["path"]
        assert np.float32(nd["split"]).view(np.uint32) == np.float32(want["split"]).view(np.uint32), \
            (want["path"], float(nd["split"]), want["split"])
        as_f32 = lambda rows: sorted(tuple(float(np.float32(v)) for v in r) for r in rows)
        assert _slot_points(p, nodes, int(nd["left"])) == as_f32(want["left"])
        assert _slot_points(p, nodes, int(nd["right"])) == as_f32(want["right"])
    check_tree(p, i, nodes, case["leaf_size"])


_OBJECT_CASES = _gold("object_median.json")["cases"]


@pytest.mark.parametrize("case", _OBJECT_CASES, ids=[c["name"] for c in _OBJECT_CASES])
def test_object_median_split_values(case):
    """Hand-derived object-median splits (Section V-C): the coordinate of rank
    floor(n/2), the fix-up when that is the minimum, and the dimension rule
    shared with the spatial median."""
    pts = np.array(case["points"], np.float32)
    p, i, nodes, h = oracle.tree_build(pts, np.arange(len(pts)), case["leaf_size"], split="object")
    for want in case["nodes"]:
        nd = nodes[_node_at(nodes, want["path"])]
        assert int(nd["dim"]) == want["dim"], want["path"]
        assert np.float32(nd["split"]).view(np.uint32) == np.float32(want["split"]).view(np.uint32), \
            (want["path"], float(nd["split"]), want["split"])
        as_f32 = lambda rows: sorted(tuple(float(np.float32(v)) for v in r) for r in rows)
        assert _slot_points(p, nodes, int(nd["left"])) == as_f32(want["left"])
        assert _slot_points(p, nodes, int(nd["right"])) == as_f32(want["right"])
    check_tree(p, i, nodes, case["leaf_size"])


@pytest.mark.parametrize("d,n,leaf", [(1, 1000, 1), (3, 5000, 16), (7, 3000, 8)])
def test_object_median_halves_distinct_coordinates(d, n, leaf):
    """With distinct coordinates the object median puts exactly floor(n/2)
    points on the left of every split, so the tree is balanced: its height is
    the one of repeated halving down to the leaf size.  A spatial-median tree
    of the same clustered points is not."""
    rng = np.random.default_rng(50 + d)
    pts = clustered_points(n, d, 60 + d, n_clusters=4)
    # make every coordinate distinct (a permutation of a fine lattice)
    for j in range(d):
        pts[np.argsort(pts[:, j], kind="stable"), j] = np.arange(n, dtype=np.float32) / n
    p, i, nodes, h = oracle.tree_build(pts, np.arange(n), leaf, split="object")
    check_tree(p, i, nodes, leaf)
    internal = nodes[nodes["dim"] >= 0]
    left_counts = nodes["count"][internal["left"]]
    assert np.array_equal(left_counts, internal["count"] // 2)
    assert np.all(nodes["count"][nodes["dim"] < 0] <= leaf)
    height, m = 1, n
    while m > leaf:
        m = m - m // 2
        height += 1
    assert h == height
    _, _, _, hs = oracle.tree_build(pts, np.arange(n), leaf, split="spatial")
    assert hs >= h


def test_object_median_log_structure_matches_bruteforce():
    """The log structure built with the object median answers k-NN like the
    definition, through inserts, erases and a half-capacity rebuild."""
    d, k = 3, 5
    o = oracle.OracleBDL(d, 4, 16, split="object")
    rng = np.random.default_rng(70)
    pts = clustered_points(3000, d, 71, n_clusters=5)
    ids = rng.permutation(10_000)[:3000].astype(np.uint32)
    live = np.zeros(3000, bool)
    for s in range(0, 3000, 500):
        o.insert(pts[s:s + 500], ids[s:s + 500])
        live[s:s + 500] = True
        e = rng.choice(np.nonzero(live)[0], 200, replace=False)
        assert o.erase(pts[e], ids[e]) == 200
        live[e] = False
        q = np.concatenate([pts[rng.choice(3000, 40)], uniform_points(40, d, s)])
        oi, od = o.knn(q, k)
        bi, bd = oracle.bruteforce_knn(pts[live], ids[live], q, k)
        assert np.array_equal(oi, bi) and np.array_equal(od.view(np.uint32), bd.view(np.uint32))
    with pytest.raises(ValueError):
        oracle.OracleBDL(d, 4, 16, split="mean")


def _tree_inputs():
    rng = np.random.default_rng(11)
    yield "uniform3", uniform_points(5000, 3, 1), 16
    yield "uniform2_leaf1", uniform_points(700, 2, 2), 1
    yield "clustered7", clustered_points(6000, 7, 3), 16
    yield "clustered3_tight", clustered_points(4000, 3, 4, n_clusters=3,
                                                log10_sigma=(-7, -6)), 8
    dup = uniform_points(50, 2, 5)
    yield "duplicates", np.repeat(dup, 40, axis=0), 16
    yield "all_same", np.full((300, 4), 0.5, np.float32), 16
    col = np.zeros((900, 3), np.float32)
    col[:, 1] = rng.random(900, dtype=np.float32)
    yield "collinear", col, 4
    neg = (rng.random((800, 2), dtype=np.float32) - 0.5) * 1e4
    neg[::7, 0] = -0.0
    neg[::11, 0] = 0.0
    yield "negative_signed_zero", neg, 16
    adj = np.array([[1.0], [np.nextafter(np.float32(1.0), np.float32(2))]], np.float32)
    yield "adjacent_floats", np.repeat(adj, 20, axis=0), 16
    yield "single", uniform_points(1, 5, 6), 16
    yield "d16", uniform_points(2000, 16, 7), 16


@pytest.mark.parametrize("name,pts,leaf", list(_tree_inputs()), ids=lambda x: x if isinstance(x, str) else "")
def test_tree_structure_invariants(name, pts, leaf):
    ids = np.arange(len(pts), dtype=np.uint32)[::-1].copy()
    p, i, nodes, h = oracle.tree_build(pts, ids, leaf)
    # slots are a permutation of the input
    order = np.argsort(i)
    assert np.array_equal(np.sort(i), np.sort(ids))
    assert np.array_equal(p[order].view(np.uint32), pts[np.argsort(ids)].view(np.uint32))
    check_tree(p, i, nodes, leaf)


def test_build_is_stable_partition():
    """Points with equal split-side keep their input order inside a leaf."""
    pts = np.zeros((40, 2), np.float32)
    pts[:, 0] = np.tile(np.array([0.0, 1.0], np.float32), 20)
    p, i, nodes, h = oracle.tree_build(pts, np.arange(40), 32)
    left = i[p[:, 0] == 0.0]
    right = i[p[:, 0] == 1.0]
    assert np.all(np.diff(left.astype(np.int64)) > 0) and np.all(np.diff(right.astype(np.int64)) > 0)
    assert np.all(p[:20, 0] == 0.0)


# --------------------------------------------------------------------------
# log structure: Insert_L
# --------------------------------------------------------------------------

def _bits(x):
    return [i for i in range(64) if (x >> i) & 1]


def test_insert_fig4_sequence():
    g = _gold("fig4_insert.json")
    X = g["X"]
    o = oracle.OracleBDL(2, leaf_size=2, buffer_size=X)
    nid = 0
    pts = uniform_points(100, 2, 9)
    o.insert(pts[:g["start_points"]], np.arange(g["start_points"]))
    nid = g["start_points"]
    info = o.level_info()
    assert info["F"] == 1 and info["buf_live"] == 0
    for st in g["steps"]:
        before = o.level_info()
        o.insert(pts[nid:nid + st["insert"]], np.arange(nid, nid + st["insert"]))
        nid += st["insert"]
        info = o.level_info()
        assert info["F"] == st["F"]
        assert info["buf_live"] == st["buffer"]
        built = [j for j in _bits(info["F"]) if not (before["F"] >> j) & 1]
        cleared = [j for j in _bits(before["F"]) if not (info["F"] >> j) & 1]
        assert built == st["built"] and cleared == st["cleared"]
        assert info["rebuilt"] - before["rebuilt"] == sum((1 << j) * X for j in st["built"])
    # the final tree 2 holds the 4X oldest points, the buffer the newest one
    ids2, _, _ = o.export_level(2)
    assert sorted(ids2.tolist()) == list(range(4 * X))
    bid, _ = o.buffer_pool()
    assert bid.tolist() == [nid - 1]


@pytest.mark.parametrize("X,seed", [(4, 0), (16, 1), (64, 2)])
def test_insert_only_binary_counter(X, seed):
    """Insert-only histories are a binary counter in units of X: F equals
    floor(n/X), the buffer holds n mod X, and each batch rebuilds exactly the
    trees whose bits turn on (Section III-C, Theorem 3's argument)."""
    rng = np.random.default_rng(seed)
    o = oracle.OracleBDL(3, leaf_size=4, buffer_size=X)
    n = 0
    F = 0
    rebuilt = 0
    for _ in range(40):
        b = int(rng.integers(0, 5 * X))
        o.insert(rng.random((b, 3), dtype=np.float32), np.arange(n, n + b))
        n += b
        Fn = n // X
        rebuilt += sum((1 << j) * X for j in _bits(Fn & ~F))
        F = Fn
        info = o.level_info()
        assert info["F"] == F and info["buf_live"] == n % X
        assert info["rebuilt"] == rebuilt
        for j in _bits(F):
            assert info["live"][j] == (1 << j) * X == info["slots"][j]
    assert o.size() == n


def test_uniform3d_10m_level_schedule_closed_form():
    """10 inserts of 1M with X = 1024 end with trees {0,2,5,9,10,13} and 640
    buffered points, and rebuild 23,520,256 points in total."""
    X = 1024
    F = 0
    n = 0
    rebuilt = 0
    for _ in range(10):
        n += 1_000_000
        Fn = n // X
        rebuilt += sum((1 << j) * X for j in _bits(Fn & ~F))
        F = Fn
    assert _bits(F) == [0, 2, 5, 9, 10, 13] and n % X == 640
    assert rebuilt == 23_520_256


# --------------------------------------------------------------------------
# log structure: Erase_L and kNN_L against bookkeeping and the definition
# --------------------------------------------------------------------------

def _collect_live(o):
    info = o.level_info()
    got = {}
    for j in _bits(info["F"]):
        ids, pts, nodes = o.export_level(j)
        check_tree(pts, ids, nodes, o.leaf_size, allow_tombstones=True)
        assert int(np.sum(ids != oracle.TOMB)) == info["live"][j]
        for i, p in zip(ids, pts):
            if i != oracle.TOMB:
                assert int(i) not in got
                got[int(i)] = p
    bids, bpts = o.buffer_pool()
    assert len(bids) == info["buf_live"] < o.buffer_size
    ex = o.export_level(-1)
    if len(bids):
        tids, tpts, tnodes = ex
        check_tree(tpts, tids, tnodes, o.leaf_size)
        assert sorted(tids.tolist()) == sorted(bids.tolist())
    for i, p in zip(bids, bpts):
        assert int(i) not in got
        got[int(i)] = p
    return got, info


@pytest.mark.parametrize("seed,d,X,leaf,clustered", [
    (0, 2, 16, 4, False), (1, 3, 32, 16, False), (2, 5, 16, 2, True), (3, 1, 16, 16, False),
    (4, 7, 64, 16, True),
])
def test_random_ops_against_bookkeeping_and_bruteforce(seed, d, X, leaf, clustered):
    o = oracle.OracleBDL(d, leaf_size=leaf, buffer_size=X)
    live = {}
    for op in random_op_sequence(seed, d, n_ops=60, max_batch=6 * X, id_capacity=1 << 20,
                                 clustered=clustered):
        if op.kind == "insert":
            o.insert(op.pts, op.ids)
            for i, p in zip(op.ids, op.pts):
                live[int(i)] = p.copy()
        elif op.kind == "erase":
            expect = 0
            seen = set()
            for i, p in zip(op.ids, op.pts):
                i = int(i)
                if i in live and i not in seen and np.array_equal(live[i].view(np.uint32), p.view(np.uint32)):
                    expect += 1
                    seen.add(i)
            got = o.erase(op.pts, op.ids)
            assert got == expect
            for i in seen:
                del live[i]
        else:
            if len(op.pts) == 0:
                continue
            ids, d2 = o.knn(op.pts, op.k)
            lid = np.array(sorted(live), np.uint32)
            lp = np.array([live[i] for i in lid], np.float32).reshape(-1, d)
            bi, bd = oracle.bruteforce_knn(lp, lid, op.pts, op.k)
            assert np.array_equal(ids, bi)
            assert np.array_equal(d2.view(np.uint32), bd.view(np.uint32))
        got, info = _collect_live(o)
        assert set(got) == set(live)
        for i, p in got.items():
            assert np.array_equal(p.view(np.uint32), live[i].view(np.uint32))
        # half-capacity rule (Alg. 4): no non-empty tree below half of 2^i X
        for j in _bits(info["F"]):
            assert 2 * info["live"][j] >= info["cap"][j]
            assert info["live"][j] <= info["cap"][j]
        assert o.size() == len(live)


def test_erased_points_never_returned_and_drain_to_empty():
    d, X = 3, 16
    o = oracle.OracleBDL(d, leaf_size=4, buffer_size=X)
    pts = uniform_points(2000, d, 3)
    ids = np.arange(2000, dtype=np.uint32)
    o.insert(pts, ids)
    rng = np.random.default_rng(3)
    order = rng.permutation(2000)
    q = uniform_points(50, d, 4)
    gone = set()
    for s in range(0, 2000, 200):
        e = order[s:s + 200]
        assert o.erase(pts[e], ids[e]) == len(e)
        gone.update(int(x) for x in ids[e])
        r, _ = o.knn(q, 7)
        assert not (set(r.ravel().tolist()) & gone)
    assert o.size() == 0
    r, dd = o.knn(q, 3)
    assert np.all(r == oracle.TOMB) and np.all(np.isinf(dd))
    assert o.level_info()["F"] == 0


def test_erase_requires_matching_coordinates():
    o = oracle.OracleBDL(2, leaf_size=4, buffer_size=8)
    pts = uniform_points(40, 2, 8)
    o.insert(pts, np.arange(40))
    bad = pts[:10].copy()
    bad[:, 1] += np.float32(0.5)
    assert o.erase(bad, np.arange(10)) == 0
    assert o.erase(pts[:10], np.arange(10) + 1000) == 0
    dup = np.concatenate([pts[:5], pts[:5]])
    assert o.erase(dup, np.concatenate([np.arange(5), np.arange(5)])) == 5
    assert o.size() == 35


def test_half_rule_fires_on_small_config():
    """Erasing about half of a full tree triggers the rebuild of Alg. 4, and
    the moved points are exactly that tree's survivors."""
    X = 16
    o = oracle.OracleBDL(2, leaf_size=4, buffer_size=X)
    pts = uniform_points(8 * X, 2, 12)
    o.insert(pts, np.arange(8 * X))
    assert o.level_info()["F"] == 8
    e = np.arange(0, 4 * X + 1)
    assert o.erase(pts[e], e) == len(e)
    info = o.level_info()
    assert info["reinserted"] == 8 * X - len(e)
    assert not (info["F"] >> 3) & 1
    got, _ = _collect_live(o)
    assert set(got) == set(range(len(e), 8 * X))


@pytest.mark.parametrize("d,leaf,X", [(2, 1, 4), (2, 2, 8), (3, 1, 4), (1, 2, 4)])
def test_tree_knn_lattice_ties_exact(d, leaf, X):
    """kNN_L on lattice points with exact ties at box boundaries: the result
    must equal the exact rational answer with ties broken by the smaller id.
    A non-strict prune (mindist^2 >= worst) drops tied points that sit in a
    subtree touching the k-th distance, and fails here."""
    rng = np.random.default_rng(40 + d + leaf)
    n = 120
    pts = rng.integers(0, 4, size=(n, d)).astype(np.float32)
    ids = rng.permutation(n).astype(np.uint32)
    o = oracle.OracleBDL(d, leaf_size=leaf, buffer_size=X)
    for s in range(0, n, 17):
        o.insert(pts[s:s + 17], ids[s:s + 17])
    q = (rng.integers(0, 7, size=(60, d)) / 2.0).astype(np.float32)
    for k in (1, 2, 3, 5, 8):
        ei, ed = _exact_knn(pts, ids, q, k)
        oi, od = o.knn(q, k)
        assert np.array_equal(oi, ei), k
        assert np.array_equal(od.astype(np.float64), ed)


def test_insert_gather_order_fig4():
    """With leaves large enough that every tree is a single leaf, a tree's
    slots are its gather order.  Reading of Alg. 3 used throughout: the
    highest new tree takes the live points of the cleared trees in ascending
    tree order, then slot order, then the leading slice of the pool (the
    buffer in arrival order followed by the batch)."""
    X = 4
    o = oracle.OracleBDL(1, leaf_size=64, buffer_size=X)
    pts = np.arange(17, dtype=np.float32).reshape(-1, 1)[::-1].copy()
    ids = np.arange(17, dtype=np.uint32)
    o.insert(pts[:4], ids[:4])
    o.insert(pts[4:9], ids[4:9])      # tree 1 = tree 0 ++ pool[0:4]; buffer [8]
    assert o.export_level(1)[0].tolist() == list(range(8))
    o.insert(pts[9:14], ids[9:14])    # tree 0 = pool[0:4] = [8, 9, 10, 11]; buffer [12, 13]
    assert o.export_level(0)[0].tolist() == [8, 9, 10, 11]
    o.insert(pts[14:17], ids[14:17])  # tree 2 = tree 0 ++ tree 1 ++ pool[0:4]
    assert o.export_level(2)[0].tolist() == [8, 9, 10, 11, 0, 1, 2, 3, 4, 5, 6, 7, 12, 13, 14, 15]
    assert o.buffer_pool()[0].tolist() == [16]


def test_parallel_knn_rows_equal_serial_rows():
    """The all-cores k-NN (queries spread over host threads) returns the
    serial oracle's rows and the same work counts."""
    d, k = 3, 5
    o = oracle.OracleBDL(d, 16, 64)
    pts = uniform_points(6000, d, 41)
    o.insert(pts, np.arange(6000, dtype=np.uint32))
    q = uniform_points(2000, d, 42)
    si, sd, sc = o.knn(q, k, counters=True)
    pi, pd, used, pc = o.knn_parallel(q, k)
    assert used >= 1
    assert np.array_equal(si, pi)
    assert np.array_equal(sd.view(np.uint32), pd.view(np.uint32))
    assert sc == pc


# --------------------------------------------------------------------------
# baselines B1 (rebuild everything) and B2 (keep the partition), Section III-B
# --------------------------------------------------------------------------

def _single_tree(o):
    info = o.level_info()
    assert info["F"] in (0, 1) and info["buf_live"] == 0
    return o.export_level(0) if info["F"] else None


def _side(ids, pts, nodes, child, live_only=False):
    nd = nodes[child]
    b, c = int(nd["begin"]), int(nd["count"])
    return sorted(tuple(float(v) for v in pts[s]) for s in range(b, b + c)
                  if not (live_only and ids[s] == oracle.TOMB))


@pytest.mark.parametrize("mode", ["rebuild_all", "no_rebuild"])
def test_baselines_fig1(mode):
    """Fig. 1: the upper tree (B1) is rebuilt around x = 4 after (5,5) and
    (7,7) arrive; the lower tree (B2) keeps its split at x = 2, puts both new
    points into the right leaf and grows that leaf's box."""
    g = _gold("fig1_baselines.json")
    o = oracle.OracleBDL(2, g["leaf_size"], 4, mode=mode)
    o.insert(np.array(g["initial"], np.float32), np.array(g["initial_ids"], np.uint32))
    o.insert(np.array(g["inserted"], np.float32), np.array(g["inserted_ids"], np.uint32))
    for stage in ("after_insert", "after_erase"):
        if stage == "after_erase":
            assert o.erase(np.array(g["erased"], np.float32), np.array(g["erased_ids"], np.uint32)) == 1
        want = g[mode][stage]
        ids, pts, nodes = _single_tree(o)
        root = nodes[0]
        assert int(root["dim"]) == want["root_dim"]
        assert np.float32(root["split"]) == np.float32(want["root_split"])
        assert _side(ids, pts, nodes, int(root["left"])) == sorted(map(tuple, map(lambda r: map(float, r), want["left"])))
        assert _side(ids, pts, nodes, int(root["right"])) == sorted(map(tuple, map(lambda r: map(float, r), want["right"])))
        r = nodes[int(root["right"])]
        if "right_box" in want:
            assert r["lo"][:2].tolist() == want["right_box"][0] and r["hi"][:2].tolist() == want["right_box"][1]
        if "root_box" in want:
            assert root["lo"][:2].tolist() == want["root_box"][0] and root["hi"][:2].tolist() == want["root_box"][1]
        if want.get("right_is_leaf"):
            assert int(r["dim"]) == -1
        if "right_live" in want:
            assert _side(ids, pts, nodes, int(root["right"]), live_only=True) == \
                sorted(map(tuple, map(lambda rr: map(float, rr), want["right_live"])))


def _check_bounding_partition(ids, pts, nodes):
    """What B2 keeps: every box bounds the points of its subtree (erased ones
    included), every point lies on its side of every split above it, and
    the leaves tile the slots."""
    covered = np.zeros(len(ids), np.int32)
    stack = [0]
    while stack:
        v = stack.pop()
        nd = nodes[v]
        b, c = int(nd["begin"]), int(nd["count"])
        sub = pts[b:b + c]
        d = pts.shape[1]
        assert np.all(sub >= nd["lo"][:d]) and np.all(sub <= nd["hi"][:d])
        if nd["dim"] < 0:
            covered[b:b + c] += 1
            continue
        l, r = nodes[int(nd["left"])], nodes[int(nd["right"])]
        assert int(l["begin"]) == b and int(l["count"]) + int(r["count"]) == c
        assert np.all(pts[b:b + int(l["count"]), int(nd["dim"])] < nd["split"])
        assert np.all(pts[b + int(l["count"]):b + c, int(nd["dim"])] >= nd["split"])
        stack += [int(nd["left"]), int(nd["right"])]
    assert np.all(covered == 1)


@pytest.mark.parametrize("mode,seed,d,clustered", [
    ("rebuild_all", 0, 2, False), ("rebuild_all", 1, 5, True),
    ("no_rebuild", 2, 2, True), ("no_rebuild", 3, 3, False), ("no_rebuild", 4, 7, True),
])
def test_baselines_random_ops(mode, seed, d, clustered):
    """Both baselines answer k-NN like the definition through random inserts
    and erases.  B1 is always one fresh build (tight boxes, leaves within the
    leaf size, nothing erased left in it); B2 never changes a split after its
    first build, keeps erased points as tombstones, and stays a bounding
    partition."""
    rng = np.random.default_rng(seed)
    leaf = 4
    o = oracle.OracleBDL(d, leaf, 16, mode=mode)
    live = {}
    splits0 = None
    ops = list(random_op_sequence(seed, d, n_ops=30, max_batch=300, id_capacity=1 << 20,
                                  clustered=clustered))
    for op in ops:
        if op.kind == "insert":
            o.insert(op.pts, op.ids)
            for p, i in zip(op.pts, op.ids):
                live[int(i)] = p
        elif op.kind == "erase":
            n0 = o.erase(op.pts, op.ids)
            hit = 0
            for p, i in zip(op.pts, op.ids):
                if int(i) in live and np.array_equal(live[int(i)].view(np.uint32), p.view(np.uint32)):
                    del live[int(i)]
                    hit += 1
            assert n0 == hit
        else:
            if op.n == 0:
                continue
            li = np.array(sorted(live), np.uint32)
            lp = np.array([live[int(i)] for i in li], np.float32).reshape(-1, d)
            oi, od = o.knn(op.pts, op.k)
            bi, bd = oracle.bruteforce_knn(lp, li, op.pts, op.k)
            assert np.array_equal(oi, bi) and np.array_equal(od.view(np.uint32), bd.view(np.uint32))
        assert o.size() == len(live)
        tr = _single_tree(o)
        if tr is None:
            continue
        ids, pts, nodes = tr
        if mode == "rebuild_all":
            assert np.all(ids != oracle.TOMB)
            check_tree(pts, ids, nodes, leaf)
        else:
            _check_bounding_partition(ids, pts, nodes)
            inner = nodes[nodes["dim"] >= 0][["dim", "split", "left", "right"]]
            if splits0 is None:
                splits0 = inner.copy()
            assert np.array_equal(inner, splits0)
    assert mode != "no_rebuild" or splits0 is not None
