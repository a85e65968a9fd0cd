"""Helpers of the GPU parity tests: run the same operations on the HIP
library and on the CPU oracle and compare results and structure."""
from __future__ import annotations

import sys

import numpy as np

TOMB = 0xFFFFFFFF
REL_TOL = 1e-6  # float32 distances must agree to 1e-6 relative


def log(msg: str) -> None:
    print(msg, flush=True)
    sys.stdout.flush()


def bits(x: int):
    return [i for i in range(64) if (x >> i) & 1]


def to_dev(a, torch, dtype=None):
    a = np.ascontiguousarray(a)
    if a.dtype == np.uint32:
        a = a.view(np.int32)
    return torch.from_numpy(a).cuda()


def assert_knn_equal(gi, gd, oi, od, what=""):
    """ids bit-exact; squared distances within 1e-6 relative and, since both
    sides evaluate the same float32 formula, bit-exact as well."""
    gi = np.asarray(gi).view(np.uint32)
    gd = np.asarray(gd, dtype=np.float32)
    assert gi.shape == oi.shape, what
    bad = np.argwhere(gi != oi)
    if bad.size:
        r = bad[0][0]
        raise AssertionError(f"{what}: {len(bad)} id mismatches; first row {r}: "
                             f"gpu {gi[r].tolist()} {gd[r].tolist()} vs oracle {oi[r].tolist()} "
                             f"{od[r].tolist()}")
    fin = np.isfinite(od)
    assert np.array_equal(np.isfinite(gd), fin), what
    rel = np.abs(gd[fin].astype(np.float64) - od[fin]) / np.maximum(np.abs(od[fin].astype(np.float64)), 1e-30)
    assert rel.size == 0 or rel.max() <= REL_TOL, f"{what}: max relative d2 error {rel.max()}"
    assert np.array_equal(gd.view(np.uint32), od.view(np.uint32)), f"{what}: d2 not bit-identical"


def compare_nodes(gn, on, d, what=""):
    assert len(gn) == len(on), f"{what}: node count gpu {len(gn)} oracle {len(on)}"
    for f in ("dim", "left", "right", "parent", "begin", "count", "depth", "path"):
        if not np.array_equal(gn[f], on[f]):
            i = int(np.argwhere(gn[f] != on[f])[0][0])
            raise AssertionError(f"{what}: node field {f} differs at node {i}: "
                                 f"gpu {gn[i]} oracle {on[i]}")
    assert np.array_equal(gn["lo"][:, :d].view(np.uint32), on["lo"][:, :d].view(np.uint32)), what
    assert np.array_equal(gn["hi"][:, :d].view(np.uint32), on["hi"][:, :d].view(np.uint32)), what
    internal = on["dim"] >= 0
    assert np.array_equal(gn["split"][internal].view(np.uint32),
                          on["split"][internal].view(np.uint32)), what


def compare_structure(tree, orc, d, what=""):
    gi = tree.level_info()
    oi = orc.level_info()
    assert gi["F"] == oi["F"], f"{what}: F gpu {gi['F']:b} oracle {oi['F']:b}"
    assert gi["buf_live"] == oi["buf_live"], what
    assert np.array_equal(gi["live"], oi["live"]), f"{what}: live {gi['live']} vs {oi['live']}"
    for j in bits(gi["F"]):
        g = tree.export_level(j)
        o = orc.export_level(j)
        assert g is not None and o is not None
        assert np.array_equal(g[0], o[0]), f"{what}: level {j} slot ids differ"
        assert np.array_equal(g[1].view(np.uint32), o[1].view(np.uint32)), f"{what}: level {j} points"
        compare_nodes(g[2], o[2], d, f"{what} level {j}")
    gb = tree.export_buffer()
    ob = orc.buffer_pool()
    assert np.array_equal(gb[0], ob[0]), f"{what}: buffer pool order"
    assert np.array_equal(gb[1].view(np.uint32), ob[1].view(np.uint32)), what
    if oi["buf_live"]:
        g = tree.export_level(-1)
        o = orc.export_level(-1)
        assert np.array_equal(g[0], o[0]), f"{what}: buffer tree slots"
        compare_nodes(g[2], o[2], d, f"{what} buffer tree")


def run_parity(tree, orc, ops, torch, d, check_structure=True, what=""):
    for n_op, op in enumerate(ops):
        tag = f"{what} op{n_op} {op.kind} n={op.n}"
        if op.kind == "insert":
            tree.insert(to_dev(op.pts, torch), to_dev(op.ids, torch))
            orc.insert(op.pts, op.ids)
        elif op.kind == "erase":
            g = tree.erase(to_dev(op.pts, torch), to_dev(op.ids, torch))
            o = orc.erase(op.pts, op.ids)
            assert g == o, f"{tag}: erased gpu {g} oracle {o}"
        else:
            if op.n == 0:
                continue
            gi, gd = tree.knn(to_dev(op.pts, torch), op.k)
            tree.sync()
            oi, od = orc.knn(op.pts, op.k)
            assert_knn_equal(gi.cpu().numpy(), gd.cpu().numpy(), oi, od, tag)
        assert tree.size() == orc.size(), tag
        if check_structure:
            compare_structure(tree, orc, d, tag)
