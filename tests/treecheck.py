"""Structural checks of one static kd-tree, written independently of both
the oracle and the GPU library.

A tree is given as points and ids in slot order and a node table in the
oracle's export layout (``oracle.NODE_DTYPE`` fields).  The checks restate
what Section III-A and Section IV-A fix about a kd-tree and its vEB layout:
children split the parent's points by an axis-aligned plane, every box is the
tight box of its points, leaves hold at most leaf_size points (coarsening,
Section V-D), and nodes are stored in van Emde Boas order (Section IV-A.1).
"""
from __future__ import annotations

import numpy as np

MAX_DEPTH = 63
TOMB = 0xFFFFFFFF


def hyperceil(x: int) -> int:
    p = 1
    while p < x:
        p <<= 1
    return p


def veb_key(H: int, depth: int, path: int) -> int:
    """Index of the node at (depth, path) in the vEB order of a complete tree
    with H levels.  A tree of l levels stores its top l_t levels first, then
    its 2^l_t bottom subtrees of l_b levels each, left to right, with
    l_b = hyperceil(floor((l+1)/2)) and l_t = l - l_b (the reading of Alg. 1
    that reproduces the worked example under Fig. 3)."""
    if H == 1:
        assert depth == 0
        return 0
    lb = hyperceil((H + 1) // 2)
    lt = H - lb
    if depth < lt:
        return veb_key(lt, depth, path)
    rel = depth - lt
    j = path >> rel
    low = path & ((1 << rel) - 1)
    return (2 ** lt - 1) + j * (2 ** lb - 1) + veb_key(lb, rel, low)


def canon(x: np.ndarray) -> np.ndarray:
    """+0 for both signed zeros (boxes hold values, not bit patterns)."""
    x = np.array(x, dtype=np.float32, copy=True)
    x[x == 0] = np.float32(0.0)
    return x


def check_tree(pts: np.ndarray, ids: np.ndarray, nodes: np.ndarray, leaf_size: int,
               allow_tombstones: bool = False) -> dict:
    """Raises AssertionError on any violation; returns a few statistics."""
    n, d = pts.shape
    nn = nodes.shape[0]
    if n == 0:
        assert nn == 0
        return {"height": 0, "leaves": 0}
    assert nn >= 1 and nn <= 2 * n - 1
    root = nodes[0]
    assert root["parent"] == -1 and root["depth"] == 0 and root["path"] == 0
    assert root["begin"] == 0 and root["count"] == n
    height = int(nodes["depth"].max()) + 1
    keys = [veb_key(height, int(nd["depth"]), int(nd["path"])) for nd in nodes]
    assert all(keys[i] < keys[i + 1] for i in range(nn - 1)), "nodes not in vEB order"
    cp = canon(pts)
    seen = np.zeros(nn, dtype=np.int64)
    leaves = 0
    covered = np.zeros(n, dtype=np.int64)
    for i in range(nn):
        nd = nodes[i]
        b, c = int(nd["begin"]), int(nd["count"])
        assert c >= 1 and 0 <= b and b + c <= n
        sub = cp[b:b + c]
        lo = sub.min(axis=0)
        hi = sub.max(axis=0)
        assert np.array_equal(nd["lo"][:d].view(np.uint32), lo.view(np.uint32)), f"box lo of node {i}"
        assert np.array_equal(nd["hi"][:d].view(np.uint32), hi.view(np.uint32)), f"box hi of node {i}"
        degenerate = bool(np.all(lo == hi))
        if nd["dim"] < 0:
            leaves += 1
            assert nd["left"] == -1 and nd["right"] == -1
            assert c <= leaf_size or degenerate or nd["depth"] >= MAX_DEPTH, f"oversized leaf {i}"
            covered[b:b + c] += 1
            continue
        assert c > leaf_size and not degenerate and nd["depth"] < MAX_DEPTH
        dim = int(nd["dim"])
        assert 0 <= dim < d
        # split dimension: depth mod d, moved forward past zero-extent dims
        c0 = int(nd["depth"]) % d
        while not hi[c0] > lo[c0]:
            c0 = (c0 + 1) % d
        assert dim == c0, f"split dim of node {i}"
        s = np.float32(nd["split"])
        assert lo[dim] < s <= hi[dim]
        L, R = int(nd["left"]), int(nd["right"])
        assert 0 <= L < nn and 0 <= R < nn
        seen[L] += 1
        seen[R] += 1
        ln, rn = nodes[L], nodes[R]
        assert ln["parent"] == i and rn["parent"] == i
        assert ln["depth"] == nd["depth"] + 1 and rn["depth"] == nd["depth"] + 1
        assert ln["path"] == (int(nd["path"]) << 1) and rn["path"] == ((int(nd["path"]) << 1) | 1)
        assert ln["begin"] == b and rn["begin"] == b + int(ln["count"])
        assert int(ln["count"]) + int(rn["count"]) == c
        assert np.all(pts[b:b + int(ln["count"]), dim] < s)
        assert np.all(pts[b + int(ln["count"]):b + c, dim] >= s)
    assert seen[0] == 0 and np.all(seen[1:] == 1), "every non-root node has one parent"
    assert np.all(covered == 1), "leaves tile the slots"
    if not allow_tombstones:
        assert not np.any(ids == TOMB)
    return {"height": height, "leaves": leaves}
