#!/usr/bin/env python3
"""Benchmark of the BDL-tree hot path on one MI355X.

A step is one pass of the whole path over the 3D workload: Insert_L of 10
batches of 1M uniform points into an empty tree, one Erase_L of 1M random
live points, then kNN_L with k = 5 for every one of the 9M live points.  All
inputs are resident in HBM before the timed region.  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "kNN queries/s + update pts/s, 10M 3D pts k=5; p50/p99 latency under mixed load"
HBM_PEAK_GBS = 8000.0


def _pct(xs, p):
    return float(np.percentile(np.asarray(xs, dtype=np.float64), p)) if xs else None


def gpu_bench(args):
    import torch

    import paper_2112_06188_amd as bdl
    from bdl_inputs import workload

    torch.cuda.set_device(0)
    w = workload(args.workload, scale=args.scale)
    dev = torch.device("cuda", 0)

    def dv(a):
        a = np.ascontiguousarray(a)
        if a.dtype == np.uint32:
            a = a.view(np.int32)
        return torch.from_numpy(a).to(dev)

    inserts = [(dv(op.pts), dv(op.ids)) for op in w.ops if op.kind == "insert"]
    erases = [(dv(op.pts), dv(op.ids)) for op in w.ops if op.kind == "erase"]
    qop = [op for op in w.ops if op.kind == "knn"][0]
    q = dv(qop.pts)
    k = qop.k
    nq = q.shape[0]
    out_ids = torch.empty((nq, k), dtype=torch.int32, device=dev)
    out_d2 = torch.empty((nq, k), dtype=torch.float32, device=dev)
    n_ins = sum(p.shape[0] for p, _ in inserts)
    n_er = sum(p.shape[0] for p, _ in erases)
    tree = bdl.Tree(w.dim, leaf_size=w.leaf_size, buffer_size=w.buffer_size,
                    id_capacity=w.id_capacity, profile=True)
    tree.set_param(bdl.PARAM_KNN_KERNEL, args.knn_kernel)
    stream = torch.cuda.current_stream(dev)
    lat = {"insert": [], "erase": [], "knn": []}

    def step(record: bool):
        tree.clear()
        evs = []
        for p, i in inserts:
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            tree.insert(p, i)
            b.record(stream)
            evs.append(("insert", a, b))
        for p, i in erases:
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            tree.erase(p, i)
            b.record(stream)
            evs.append(("erase", a, b))
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        tree.knn(q, k, out_ids, out_d2)
        b.record(stream)
        evs.append(("knn", a, b))
        if record:
            torch.cuda.synchronize()
            for kind, a, b in evs:
                lat[kind].append(a.elapsed_time(b))

    for _ in range(args.warmup):
        step(False)
    tree.sync()
    tree.profile(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    tree.sync()
    prof = tree.profile()
    elapsed = t1 - t0
    ms_step = elapsed * 1e3 / args.steps

    # full-size property check: every query is a live point, so its own id is
    # its nearest neighbour at squared distance 0 (no duplicate coordinates)
    qids = dv(np.nonzero(np.isin(np.arange(w.id_capacity), np.asarray(
        [op.ids for op in w.ops if op.kind == "erase"][0]), invert=True))[0].astype(np.uint32))
    self_ok = bool(torch.equal(out_ids[:, 0], qids)) and bool((out_d2[:, 0] == 0).all())

    info = tree.level_info()
    sizes = tree.level_sizes()
    S = (w.dim + 1 + 3) & ~3
    NS = (5 + 2 * w.dim + 3) & ~3
    tree_bytes = int(sizes["slots"].sum()) * S * 4 + int(sizes["nodes"].sum()) * NS * 4
    tree_bytes += info["buf_live"] * S * 4 + sizes["buf_nodes"] * NS * 4
    trav = prof["traverse"]
    trav_ms = trav["ms"] / max(1, trav["calls"])
    # algorithmic bytes of one traversal launch: queries read, the Morton
    # order read, results written, every live tree read once
    alg_bytes = nq * (4 * w.dim + 4 + 8 * k) + tree_bytes
    achieved = alg_bytes / (trav_ms * 1e-3) / 1e9
    ins_ms = float(np.sum(lat["insert"])) / args.steps
    er_ms = float(np.sum(lat["erase"])) / args.steps
    knn_ms = float(np.sum(lat["knn"])) / args.steps
    res = {
        "metric": METRIC,
        "value": (n_ins + n_er + nq) / (ms_step * 1e-3),
        "unit": "ops/s (inserted + erased points + kNN queries per second)",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded uniform float32 points in [0,1)^3)",
        "config": {"workload": w.name, "n_points": n_ins, "dim": w.dim, "k": k,
                   "knn_kernel": ["lane", "wave"][args.knn_kernel],
                   "insert_batches": len(inserts), "erase_points": n_er, "queries": nq,
                   "leaf_size": w.leaf_size, "buffer_size": w.buffer_size},
        "knn_queries_per_s": nq / (knn_ms * 1e-3),
        "insert_pts_per_s": n_ins / (ins_ms * 1e-3),
        "erase_pts_per_s": n_er / (er_ms * 1e-3),
        "latency_ms": {kind: {"p50": _pct(v, 50), "p99": _pct(v, 99), "n": len(v)}
                       for kind, v in lat.items()},
        "phase_ms_per_step": {kname: v["ms"] / args.steps for kname, v in prof.items()
                              if kname != "knn_work"},
        "knn_work_per_query": {kname: v / (args.steps * nq) for kname, v in prof["knn_work"].items()},
        "final_levels": [i for i in range(64) if (info["F"] >> i) & 1],
        "buffer_points": info["buf_live"],
        "self_match_all_queries": self_ok,
        "roofline": {"kernel": "k_knn (kNN_L traversal)", "bound": "hbm",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "algorithmic_bytes_per_launch": alg_bytes,
                     "avg_launch_ms": trav_ms},
    }
    tree.close()
    return res, w, (q, out_ids, out_d2)


def cpu_baseline(w, gpu_out, n_sample: int):
    """The oracle on the host: the full update sequence, then kNN_L on a
    sample of the queries; throughput in the benchmark's unit (the kNN time
    is scaled from the sample to all queries)."""
    import oracle

    o = oracle.OracleBDL(w.dim, w.leaf_size, w.buffer_size)
    t_ins = t_er = 0.0
    n_ins = n_er = 0
    for op in w.ops:
        if op.kind == "insert":
            t0 = time.perf_counter()
            o.insert(op.pts, op.ids)
            t_ins += time.perf_counter() - t0
            n_ins += op.n
        elif op.kind == "erase":
            t0 = time.perf_counter()
            o.erase(op.pts, op.ids)
            t_er += time.perf_counter() - t0
            n_er += op.n
    qop = [op for op in w.ops if op.kind == "knn"][0]
    nq = qop.n
    sel = np.random.default_rng(123).choice(nq, size=min(n_sample, nq), replace=False)
    sel.sort()
    t0 = time.perf_counter()
    oi, od = o.knn(qop.pts[sel], qop.k)
    t_knn = time.perf_counter() - t0
    # parity on the sample at full size
    q, gi, gd = gpu_out
    g_ids = gi.cpu().numpy().view(np.uint32)[sel]
    g_d2 = gd.cpu().numpy()[sel]
    ids_equal = bool(np.array_equal(g_ids, oi))
    d2_equal = bool(np.array_equal(g_d2.view(np.uint32), od.view(np.uint32)))
    t_total = t_ins + t_er + t_knn * nq / len(sel)
    return {
        "value": (n_ins + n_er + nq) / t_total,
        "unit": "ops/s (inserted + erased points + kNN queries per second)",
        "cores": 1,
        "kind": "oracle",
        "sample": (f"serial oracle: all {len(w.ops) - 2} inserts and the erase at full size, "
                   f"kNN_L on {len(sel)} of {nq} queries (time scaled to all queries)"),
        "insert_pts_per_s": n_ins / t_ins,
        "erase_pts_per_s": n_er / t_er,
        "knn_queries_per_s": len(sel) / t_knn,
        "seconds": t_ins + t_er + t_knn,
        "host": {"nproc": os.cpu_count(), "cpu": platform.processor() or platform.machine()},
        "gpu_matches_oracle_on_sample": {"ids": ids_equal, "d2_bitwise": d2_equal},
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="uniform3d_10m")
    ap.add_argument("--scale", type=float, default=1.0)
    ap.add_argument("--knn-kernel", type=int, default=1, choices=[0, 1],
                    help="0: one lane per query, 1: one wavefront per 64 queries")
    ap.add_argument("--cpu-sample", type=int, default=200_000,
                    help="queries the CPU oracle answers for the baseline (0: skip)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(see DESIGN.md for how the structure would shard)", file=sys.stderr)
        sys.exit(2)
    res, w, gpu_out = gpu_bench(args)
    if args.cpu_sample > 0:
        res["cpu_baseline"] = cpu_baseline(w, gpu_out, args.cpu_sample)
    else:
        res["cpu_baseline"] = None
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
