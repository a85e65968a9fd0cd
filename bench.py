#!/usr/bin/env python3
"""Benchmark of the BDL-tree hot path on one MI355X.

Default form (plain): a step is one pass of the whole path over the 3D
workload: Insert_L of 10 batches of 1M uniform points into an empty tree,
one Erase_L of 1M random live points, then kNN_L with k = 5 for every one of
the 9M live points.  All inputs are resident in HBM before the timed region.
Prints one JSON line.

--form batched: the op log of 4096 uneven 5D kNN_L batches (k in {1,5,10})
and 128 Insert_L batches over a 20M-point resident set, run once call by
call (bdl_knn per batch) and once in the batched form (bdl_knn_batch over
the kNN batches between two inserts, replayed hipGraphs), both with the
autotuned launch shapes; results must be identical.

--form mixed: the mixed-operations experiment of Section VI-D.3 (20 inserts
and 15 erases of 5% each, kNN_L over every live point after every fifth)
on the BDL-tree and the baselines B1 (rebuild all) and B2 (no rebuild).

--form served: a 50M-point 3D clustered resident set and 2000 requests
(70% kNN_L k=5, 20% Insert_L, 10% Erase_L) arriving as a Poisson stream at
0.5, 0.8 and 0.95 of the FIFO loop's saturation rate, served by the native
request loop in FIFO mode and with continuous batching; p50/p99 latency and
throughput of both, and the k-NN results of the two compared.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--form plain|batched|served|mixed]
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
# FP32 vector FMA rate without packed-FP32 instructions (256 CUs x 2.4 GHz x
# 128 flops per CU per clock); the library is built with packed FP32 off, so
# this is the rate its kernels can reach (157.3 TFLOP/s needs packed FP32)
FP32_PEAK_TFLOPS = 78.6
# HBM traffic of the traversal kernel measured with rocprofv3 counters
# (FETCH_SIZE, WRITE_SIZE) and the sources it was measured on
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "knn_traversal_traffic.json")
TRAVERSAL_SOURCES = [os.path.join(ROOT, "paper_2112_06188_amd", "csrc", f)
                     for f in ("knn_traverse.hpp", "knn_d1_4.hip", "knn.hip")]


def traversal_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in TRAVERSAL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic():
    """Bytes per traversal launch from the committed counter measurement, or
    None when there is none or the kernel's sources changed since."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("source_sha256") != traversal_source_hash():
        return None
    return t.get("bytes_per_launch")


def _pct(xs, p):
    return float(np.percentile(np.asarray(xs, dtype=np.float64), p)) if xs else None


def traversal_kernel(mode: int, d: int, nq: int, live: int) -> str:
    """The traversal kernel a plain bdl_knn launch runs (BDL_PARAM_KNN_KERNEL;
    2 is the library's default choice for one launch of nq queries)."""
    if mode == 2:
        if d >= 5 or nq <= 131072:
            mode = 3
        else:
            mode = 1 if (nq >= 65536 and 2 * nq >= live) else 0
    return {0: "k_knn", 1: "k_knn_wave", 3: "k_knn_query"}[mode]


def knn_graph_leg(torch, bdl, tree, out_ids, out_d2, qids, k, stream):
    """The step's k-NN rows (every live point as a query) through
    bdl_knn_graph, both ways: presorted queries searched from the roots, and
    the leaf-based search of Section II (one wavefront per subtree, starting
    there).  Device time of the whole call against the step's kNN_L, and the
    rows compared with kNN_L's bit for bit."""
    gi = torch.empty((tree.id_capacity, k), dtype=torch.int32, device=out_ids.device)
    gd = torch.empty((tree.id_capacity, k), dtype=torch.float32, device=out_ids.device)
    rows = qids.to(torch.int64)
    nq = qids.shape[0]
    out = {}
    for name, start in (("presorted", 0), ("leaf_based", 1)):
        tree.set_param(bdl.PARAM_GRAPH_START, start)
        ms = []
        tree.sync()
        tree.profile(reset=True)
        for _ in range(3):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            tree.knn_graph(k, gi, gd)
            b.record(stream)
            torch.cuda.synchronize()
            ms.append(a.elapsed_time(b))
        same = bool(torch.equal(gi[rows], out_ids)) and \
            bool(torch.equal(gd[rows].view(torch.int32), out_d2.view(torch.int32)))
        t = float(np.median(ms))
        tree.sync()
        prof = tree.profile(reset=True)
        out[name] = {"ms": t, "queries_per_s": nq / (t * 1e-3), "calls_ms": ms,
                     "gather_or_groups_and_order_ms": prof["order"]["ms"] / 3,
                     "traverse_ms": prof["traverse"]["ms"] / 3,
                     "work_per_query": {kk: v / (3 * nq) for kk, v in prof["knn_work"].items()},
                     "rows_equal_knn": same}
    tree.set_param(bdl.PARAM_GRAPH_START, 0)
    del gi, gd
    return out


def erase_route_leg(torch, bdl, tree, inserts, erases, stream):
    """The step's erases located through the id map and, as Erase_S with
    per-tree Bloom filters (Section V-A), by routing each point down the
    trees; the routed time includes building the filters (lazily, at the
    first erase after the trees changed).  Untimed inserts before each."""
    out = {}
    counts = {}
    n_er = sum(p.shape[0] for p, _ in erases)
    for name, route in (("map", 0), ("routed", 1)):
        tree.set_param(bdl.PARAM_ERASE_ROUTE, route)
        ms = []
        for rep in range(2):
            tree.clear()
            for p, i in inserts:
                tree.insert(p, i)
            tree.sync()
            got = []
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            for p, i in erases:
                got.append(tree.erase(p, i))
            b.record(stream)
            torch.cuda.synchronize()
            ms.append(a.elapsed_time(b))
        counts[name] = got
        out[name] = {"ms": ms[-1], "pts_per_s": n_er / (ms[-1] * 1e-3)}
    tree.set_param(bdl.PARAM_ERASE_ROUTE, 0)
    out["same_counts"] = counts["map"] == counts["routed"]
    return out


def gpu_bench(args):
    import torch

    import paper_2112_06188_amd as bdl
    from bdl_inputs import workload

    torch.cuda.set_device(0)
    w = workload(args.workload, scale=args.scale)
    dev = torch.device("cuda", 0)
    if args.copy_probe_mib:
        # a plain copy of known size, for scaling the HBM counters of a
        # profiled run (reads and writes copy_probe_mib MiB once)
        n = args.copy_probe_mib << 18
        a = torch.ones(n, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        torch.mul(a, 1.0, out=b)
        torch.cuda.synchronize()
        del a, b

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
    route_leg = erase_route_leg(torch, bdl, tree, inserts, erases, stream) if args.extra else None

    # full-size property check: every query is a live point (queries in
    # ascending id order), so each row starts at squared distance 0 with its
    # own id, or with a smaller id at the same coordinates
    qids = dv(np.nonzero(np.isin(np.arange(w.id_capacity), np.asarray(
        [op.ids for op in w.ops if op.kind == "erase"][0]), invert=True))[0].astype(np.uint32))
    first = out_ids[:, 0].to(torch.int64) & 0xFFFFFFFF
    own = qids.to(torch.int64) & 0xFFFFFFFF
    self_ok = bool((out_d2[:, 0] == 0).all()) and bool((first <= own).all())
    self_exact = float((first == own).to(torch.float32).mean())
    graph_leg = knn_graph_leg(torch, bdl, tree, out_ids, out_d2, qids, k, stream) \
        if args.extra \
        else None
    counters = tree.counters()

    info = tree.level_info()
    sizes = tree.level_sizes()
    bdl_live = int(info["live"].sum()) + int(info["buf_live"])
    S = (w.dim + 1 + 3) & ~3
    NS = (5 + 2 * w.dim + 3) & ~3
    tree_bytes = int(sizes["slots"].sum()) * S * 4 + int(sizes["nodes"].sum()) * NS * 4
    tree_bytes += info["buf_live"] * S * 4 + sizes["buf_nodes"] * NS * 4
    trav = prof["traverse"]
    trav_ms = trav["ms"] / max(1, trav["calls"])
    # algorithmic bytes of one traversal launch: queries read, the Hilbert
    # order read, results written, every live tree read once
    alg_bytes = nq * (4 * w.dim + 4 + 8 * k) + tree_bytes
    achieved = alg_bytes / (trav_ms * 1e-3) / 1e9
    work = prof["knn_work"]
    valu_flops = float(work["points"] * 3 * w.dim + work["nodes"] * 5 * w.dim) / max(1, args.steps)
    ins_ms = float(np.sum(lat["insert"])) / args.steps
    # compulsory HBM bytes of the step's Insert_L calls: every batch read once,
    # every rebuilt point gathered (read) and written to its tree once, and the
    # rebuilt trees' nodes written once (node count estimated from the final
    # trees' nodes per slot)
    rebuilt = counters["rebuilt"]
    nodes_per_slot = (int(sizes["nodes"].sum()) / max(1, int(sizes["slots"].sum())))
    ins_bytes = n_ins * 4 * (w.dim + 1) + rebuilt * 2 * 4 * (w.dim + 1) + \
        int(rebuilt * nodes_per_slot) * NS * 4
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
                   "knn_kernel": ["lane", "wave", "auto"][args.knn_kernel],
                   "insert_batches": len(inserts), "erase_points": n_er, "queries": nq,
                   "leaf_size": w.leaf_size, "buffer_size": w.buffer_size},
        "knn_queries_per_s": nq / (knn_ms * 1e-3),
        "insert_pts_per_s": n_ins / (ins_ms * 1e-3),
        "erase_pts_per_s": n_er / (er_ms * 1e-3),
        "erase_route": route_leg,
        "knn_graph": graph_leg,
        "sequential_call_latency_ms": {kind: {"p50": _pct(v, 50), "p99": _pct(v, 99), "n": len(v)}
                       for kind, v in lat.items()},
        "phase_ms_per_step": {kname: v["ms"] / args.steps for kname, v in prof.items()
                              if kname != "knn_work"},
        "knn_work_per_query": {kname: v / (args.steps * nq) for kname, v in prof["knn_work"].items()},
        "final_levels": [i for i in range(64) if (info["F"] >> i) & 1],
        "buffer_points": info["buf_live"],
        "self_match_all_queries": self_ok,
        "self_match_own_id_fraction": self_exact,
        "insert_roofline": {"bound": "hbm", "compulsory_bytes_per_step": ins_bytes,
                            "rebuilt_points_per_step": rebuilt,
                            "insert_ms_per_step": ins_ms,
                            "achieved": ins_bytes / (ins_ms * 1e-3) / 1e9,
                            "peak": HBM_PEAK_GBS, "unit": "GB/s",
                            "frac": ins_bytes / (ins_ms * 1e-3) / 1e9 / HBM_PEAK_GBS},
        "roofline": {"kernel": traversal_kernel(args.knn_kernel, w.dim, nq, bdl_live)
                     + " (kNN_L traversal)", "bound": "hbm",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(),
                     "algorithmic_bytes_per_launch": alg_bytes,
                     "avg_launch_ms": trav_ms,
                     # the same launch against the FP32 vector peak: flops of
                     # the distance evaluations (sub + fma per coordinate) and
                     # box tests (two subs, a select and an fma per
                     # coordinate) the GPU counted
                     "valu": {"achieved": valu_flops / (trav_ms * 1e-3) / 1e12,
                              "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                              "frac": valu_flops / (trav_ms * 1e-3) / 1e12 / FP32_PEAK_TFLOPS,
                              "flops_per_launch": valu_flops}},
    }
    tree.close()
    return res, w, (q, out_ids, out_d2)


def _dv(torch, a):
    a = np.ascontiguousarray(a)
    if a.dtype == np.uint32:
        a = a.view(np.int32)
    return torch.from_numpy(a).to("cuda")


def batched_bench(args):
    """Plain per-call path vs the batched form on the same op log."""
    import torch

    import paper_2112_06188_amd as bdl
    from bdl_inputs import uniform_points, workload
    from paper_2112_06188_amd import autotune

    torch.cuda.set_device(0)
    w = workload("batched5d_20m", scale=args.scale)
    setup = [(_dv(torch, op.pts), _dv(torch, op.ids)) for op in w.ops[:w.n_setup]]
    log = []
    for op in w.ops[w.n_setup:]:
        if op.kind == "knn":
            log.append(("knn", _dv(torch, op.pts), op.k))
        else:
            log.append(("insert", _dv(torch, op.pts), _dv(torch, op.ids)))
    n_q = sum(x[1].shape[0] for x in log if x[0] == "knn")
    n_ins = sum(x[1].shape[0] for x in log if x[0] == "insert")
    n_kb = sum(1 for x in log if x[0] == "knn")

    def outputs():
        return [(torch.empty((x[1].shape[0], x[2]), dtype=torch.int32, device="cuda"),
                 torch.empty((x[1].shape[0], x[2]), dtype=torch.float32, device="cuda"))
                if x[0] == "knn" else None for x in log]

    out_plain, out_batch = outputs(), outputs()
    tree = bdl.Tree(w.dim, leaf_size=w.leaf_size, buffer_size=w.buffer_size,
                    id_capacity=w.id_capacity)

    def build_resident():
        tree.clear()
        for p, i in setup:
            tree.insert(p, i)
        tree.sync()

    build_resident()
    # launch shapes: tuned on the resident set with fresh queries (not timed)
    tq = _dv(torch, uniform_points(1 << 20, w.dim, 999))
    t0 = time.perf_counter()
    tuned = autotune.tune(tree, lambda n: tq[:n], k_bands=((1, 1), (2, 5), (6, 10)),
                          nq_bands=((1, 2048), (2049, 32768), (32769, 262144),
                                    (262145, 1 << 40)),
                          max_nq=1 << 20, reps=2,
                          cands=autotune.candidates(blocks=(64, 256)),
                          log=lambda m: print(f"batched: tune {m}", file=sys.stderr, flush=True))
    tune_s = time.perf_counter() - t0
    stream = torch.cuda.current_stream()

    def timed_insert(x, ins):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        tree.insert(x[1], x[2])
        b.record(stream)
        ins.append((a, b))

    def run_plain():
        lat, ins = [], []
        for x, o in zip(log, out_plain):
            if x[0] == "knn":
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record(stream)
                tree.knn(x[1], x[2], o[0], o[1])
                b.record(stream)
                lat.append((a, b))
            else:
                timed_insert(x, ins)
        return lat, ins

    def run_batched():
        pend, po, ins = [], [], []
        for x, o in zip(log, out_batch):
            if x[0] == "knn":
                pend.append((x[1], x[2]))
                po.append(o)
            else:
                if pend:
                    tree.knn_batch(pend, po)
                    pend, po = [], []
                timed_insert(x, ins)
        if pend:
            tree.knn_batch(pend, po)
        return [], ins

    res = {}
    for name, fn in (("plain", run_plain), ("batched", run_batched)):
        for _ in range(args.warmup):
            build_resident()
            fn()
            tree.sync()
        times, lats, ins_s = [], [], []
        for _ in range(args.steps):
            build_resident()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            lat, ins = fn()
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
            tree.sync()
            lats += [a.elapsed_time(b) for a, b in lat]
            ins_s.append(sum(a.elapsed_time(b) for a, b in ins) / 1e3)
        sec = float(np.median(times))
        ins_sec = float(np.median(ins_s))
        print(f"batched: {name} {sec:.3f} s (inserts {ins_sec:.3f} s)", file=sys.stderr, flush=True)
        res[name] = {"seconds": sec, "ops_per_s": (n_q + n_ins) / sec,
                     "insert_seconds": ins_sec,
                     "knn_queries_per_s": n_q / max(1e-9, sec - ins_sec)}
        if lats:
            res[name]["knn_call_latency_ms"] = {"p50": _pct(lats, 50), "p99": _pct(lats, 99)}
    same = all(torch.equal(a[0], b[0]) and torch.equal(a[1].view(torch.int32), b[1].view(torch.int32))
               for a, b in zip(out_plain, out_batch) if a is not None)
    # sampled parity against the definition: 2 queries of every 64th kNN
    # batch, brute force over the live set at that point of the log
    check = None
    if args.cpu_sample > 0:
        import oracle
        # the workload's points are one array in insertion order and nothing
        # is erased, so the live set at any point of the log is a prefix
        allp = np.concatenate([op.pts for op in w.ops if op.kind == "insert"])
        alli = np.concatenate([op.ids for op in w.ops if op.kind == "insert"])
        n_live = sum(op.n for op in w.ops[:w.n_setup])
        ok = True
        nchk = 0
        t0 = time.perf_counter()
        kb = 0
        for op, o in zip(w.ops[w.n_setup:], out_batch):
            if op.kind == "insert":
                n_live += op.n
                continue
            if kb % 64 == 0:
                sel = np.unique(np.array([0, op.n - 1]))
                oi, od = oracle.bruteforce_knn(allp[:n_live], alli[:n_live], op.pts[sel], op.k)
                gi = o[0].cpu().numpy().view(np.uint32)[sel]
                gd = o[1].cpu().numpy()[sel]
                ok &= bool(np.array_equal(gi, oi) and
                           np.array_equal(gd.view(np.uint32), od.view(np.uint32)))
                nchk += len(sel)
            kb += 1
        check = {"queries_checked": nchk, "equal_to_bruteforce": ok,
                 "seconds": time.perf_counter() - t0}
    tree.close()
    sp = res["plain"]["seconds"] / res["batched"]["seconds"]
    return {
        "metric": "batched form vs plain path: kNN_L + Insert_L ops/s on one op log "
                  "(4096 uneven 5D kNN batches, 128 inserts, 20M resident)",
        "value": res["batched"]["ops_per_s"],
        "unit": "ops/s (kNN queries + inserted points per second)",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": res["batched"]["seconds"] * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded uniform float32 points in [0,1)^5)",
        "config": {"workload": w.name, "dim": w.dim, "knn_batches": n_kb, "queries": n_q,
                   "insert_batches": len(log) - n_kb, "inserted_points": n_ins,
                   "resident_points": sum(p.shape[0] for p, _ in setup)},
        "plain": res["plain"], "batched": res["batched"],
        "speedup_batched_over_plain": sp,
        "results_identical": same,
        "oracle_check": check,
        "autotune": {"seconds": tune_s, "rows": tuned["rows"]},
    }


def served_bench(args, scale=None, lambdas=(0.5, 0.8, 0.95)):
    """FIFO loop vs continuous batching on one Poisson request stream."""
    import torch

    import paper_2112_06188_amd as bdl
    from bdl_inputs import workload

    torch.cuda.set_device(0)
    t_gen = time.perf_counter()
    w = workload("served3d_50m", scale=args.scale if scale is None else scale)
    t_gen = time.perf_counter() - t_gen
    setup = [(_dv(torch, op.pts), _dv(torch, op.ids)) for op in w.ops[:w.n_setup]]
    reqs = w.ops[w.n_setup:]
    tree = bdl.Tree(w.dim, leaf_size=w.leaf_size, buffer_size=w.buffer_size,
                    id_capacity=w.id_capacity)

    def rebuild():
        tree.clear()
        for p, i in setup:
            tree.insert(p, i)
        tree.sync()

    rebuild()
    budget = int(torch.cuda.mem_get_info()[0] // 2)
    print(f"served: {w.description}; staging budget {budget >> 20} MiB", file=sys.stderr,
          flush=True)

    def run(mode, rate, seed=5):
        rebuild()
        srv = bdl.Server(tree, mode=mode, max_inflight=4096, max_batch_requests=4096,
                         max_batch_queries=1 << 22, max_launches=2, mem_budget=budget)
        n = len(reqs)
        if rate:
            at = np.cumsum(np.random.default_rng(seed).exponential(1.0 / rate, size=n))
        else:
            at = np.zeros(n)
        tickets = []
        t0 = time.perf_counter()
        for a, op in zip(at, reqs):
            while True:
                dt = t0 + a - time.perf_counter()
                if dt <= 0:
                    break
                time.sleep(dt if dt > 2e-3 else 0)
            if len(tickets) % 500 == 499:
                print(f"served: {len(tickets) + 1} submitted at {time.perf_counter() - t0:.1f} s",
                      file=sys.stderr, flush=True)
            if op.kind == "knn":
                tickets.append(srv.submit_knn(op.pts, op.k))
            elif op.kind == "insert":
                tickets.append(srv.submit_insert(op.pts, op.ids))
            else:
                tickets.append(srv.submit_erase(op.pts, op.ids))
        comps = [srv.wait(tk) for tk in tickets]
        srv.close()
        lat = np.array([c["t_done_ms"] - c["t_submit_ms"] for c in comps])
        klat = np.array([c["t_done_ms"] - c["t_submit_ms"] for c in comps if c["kind"] == 0])
        span_s = (max(c["t_done_ms"] for c in comps) - min(c["t_submit_ms"] for c in comps)) / 1e3
        st = {"requests_per_s": n / span_s, "seconds": span_s,
              "latency_ms": {"p50": float(np.percentile(lat, 50)),
                             "p99": float(np.percentile(lat, 99))},
              "knn_latency_ms": {"p50": float(np.percentile(klat, 50)),
                                 "p99": float(np.percentile(klat, 99))},
              "launches": int(len({c["launch"] for c in comps})),
              "failed": int(sum(c["status"] != 0 for c in comps))}
        if rate:
            st["offered_requests_per_s"] = rate
        print(f"served: mode {mode} rate {rate}: {json.dumps(st)}", file=sys.stderr, flush=True)
        return st, comps

    out = {}
    print("served: saturation runs", file=sys.stderr, flush=True)
    sat_fifo, comps_fifo = run(bdl.SERVE_FIFO, None)
    sat_bat, comps_bat = run(bdl.SERVE_BATCHED, None)
    same = all(np.array_equal(a["ids"], b["ids"]) and
               np.array_equal(a["d2"].view(np.uint32), b["d2"].view(np.uint32))
               for a, b in zip(comps_fifo, comps_bat) if a["kind"] == 0)
    erased_same = all(a["n_erased"] == b["n_erased"] for a, b in zip(comps_fifo, comps_bat))
    del comps_fifo, comps_bat
    out["saturation"] = {"fifo": sat_fifo, "batched": sat_bat}
    rate = sat_fifo["requests_per_s"]
    for lam in lambdas:
        row = {}
        for name, mode in (("fifo", bdl.SERVE_FIFO), ("batched", bdl.SERVE_BATCHED)):
            print(f"served: lambda {lam} {name}", file=sys.stderr, flush=True)
            row[name], _ = run(mode, lam * rate)
        out[f"lambda_{lam}"] = row
    tree.close()
    hi = out[f"lambda_{lambdas[-1]}"]
    return {
        "metric": "served form: request throughput and p50/p99 latency under a Poisson "
                  "stream (3D clustered, 50M resident, 70/20/10 kNN/insert/erase)",
        "value": sat_bat["requests_per_s"],
        "unit": "requests/s (saturation, continuous batching)",
        "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": sat_bat["seconds"] * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded 3D Gaussian-blob mixture, float32)",
        "config": {"workload": w.name, "requests": len(reqs),
                   "resident_points": sum(p.shape[0] for p, _ in setup),
                   "staging_budget_bytes": budget},
        "saturation_speedup_batched_over_fifo":
            sat_bat["requests_per_s"] / sat_fifo["requests_per_s"],
        f"p99_ratio_fifo_over_batched_at_{lambdas[-1]}": hi["fifo"]["latency_ms"]["p99"] /
            hi["batched"]["latency_ms"]["p99"],
        "results_identical_fifo_vs_batched": bool(same and erased_same),
        "runs": out,
        "generation_seconds": t_gen,
    }


def mixed_bench(args, name=None, scale=None):
    """The mixed-operations experiment of Section VI-D.3 on the BDL-tree and
    on the two baselines of Section III-B (B1 rebuilds its one tree after
    every update, B2 never does): per section (five updates, then kNN_L for
    every live point) the update and k-NN device times; the three structures
    must return identical k-NN rows."""
    import torch

    import paper_2112_06188_amd as bdl
    from bdl_inputs import workload

    torch.cuda.set_device(0)
    w = workload(name or args.mixed_workload, scale=args.scale if scale is None else scale)
    stream = torch.cuda.current_stream()
    ops = []
    for op in w.ops:
        if op.kind == "knn":
            ops.append(("knn", _dv(torch, op.pts), op.k))
        else:
            ops.append((op.kind, _dv(torch, op.pts), _dv(torch, op.ids)))
    labels = ["INS0", "INS1", "INS2", "INS3", "DEL0", "DEL1", "DEL2"]
    ref = None
    out = {}
    for structure in ("bdl", "rebuild_all", "no_rebuild"):
        tree = bdl.Tree(w.dim, leaf_size=w.leaf_size, buffer_size=w.buffer_size,
                        id_capacity=w.id_capacity, structure=structure)
        evs, results, sec = [], [], 0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for kind, x, y in ops:
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            if kind == "insert":
                tree.insert(x, y)
            elif kind == "erase":
                tree.erase(x, y)
            else:
                results.append(tree.knn(x, y))
            b.record(stream)
            evs.append((kind, sec, a, b))
            if kind == "knn":
                sec += 1
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        tree.sync()
        secs = [{"section": labels[i], "update_ms": 0.0, "knn_ms": 0.0} for i in range(sec)]
        for kind, i, a, b in evs:
            secs[i]["knn_ms" if kind == "knn" else "update_ms"] += a.elapsed_time(b)
        for r in secs:
            r["total_ms"] = r["update_ms"] + r["knn_ms"]
        same = None
        if ref is None:
            ref = results
        else:
            same = all(torch.equal(p[0], q[0]) and torch.equal(p[1].view(torch.int32),
                                                             q[1].view(torch.int32))
                       for p, q in zip(ref, results))
        if ref is not results:
            del results
        tree.close()
        out[structure] = {"sections": secs, "wall_seconds": wall,
                          "update_ms": sum(r["update_ms"] for r in secs),
                          "knn_ms": sum(r["knn_ms"] for r in secs),
                          "total_ms": sum(r["total_ms"] for r in secs),
                          "knn_rows_equal_to_bdl": same}
        print(f"mixed: {structure} total {out[structure]['total_ms']:.1f} ms "
              f"(updates {out[structure]['update_ms']:.1f}, knn {out[structure]['knn_ms']:.1f})",
              file=sys.stderr, flush=True)
    best = min(out, key=lambda kk: out[kk]["total_ms"])
    # sampled rows of the last k-NN pass against brute force over the live set
    check = None
    if args.cpu_sample > 0:
        import oracle
        q = ops[-1][1].cpu().numpy()
        sel = np.sort(np.random.default_rng(3).choice(q.shape[0], 16, replace=False))
        dead = np.concatenate([op.ids for op in w.ops if op.kind == "erase"])
        live = np.ones(w.id_capacity, bool)
        live[dead.astype(np.int64)] = False
        allp = np.concatenate([op.pts for op in w.ops if op.kind == "insert"])
        oi, od = oracle.bruteforce_knn(allp[live], np.nonzero(live)[0].astype(np.uint32), q[sel], 5)
        gi = ref[-1][0].cpu().numpy().view(np.uint32)[sel]
        gd = ref[-1][1].cpu().numpy()[sel]
        check = {"rows": len(sel), "equal": bool(np.array_equal(gi, oi) and
                                                 np.array_equal(gd.view(np.uint32), od.view(np.uint32)))}
    return {
        "metric": "mixed operations (Section VI-D.3): device time of 20 inserts, 15 erases and "
                  "7 k-NN passes over every live point, BDL-tree vs baselines B1 and B2",
        "value": out["bdl"]["total_ms"], "unit": "ms (whole experiment, BDL-tree)",
        "higher_is_better": False, "n_gpus": 1, "dtype": "f32",
        "data": f"synthetic ({w.description})",
        "config": {"workload": w.name, "dim": w.dim, "points": w.id_capacity,
                   "leaf_size": w.leaf_size, "buffer_size": w.buffer_size},
        "structures": out, "best_total": best,
        "speedup_bdl_over_rebuild_all": out["rebuild_all"]["total_ms"] / out["bdl"]["total_ms"],
        "speedup_bdl_over_no_rebuild": out["no_rebuild"]["total_ms"] / out["bdl"]["total_ms"],
        "bruteforce_rows": check,
    }


def served_leg(args):
    """The metric's mixed-load half: the served form on the clustered 3D
    request stream with a 10M-point resident set (the served workload at
    scale 0.2: 2000 requests, 70% kNN_L k=5 of 1-65536 queries, 20% Insert_L
    and 10% Erase_L of 200-200K points), Poisson arrivals at 0.5 and 0.8 of
    the FIFO loop's saturation rate; p50/p99 latency of the FIFO loop and of
    continuous batching, whose results must be identical."""
    r = served_bench(args, scale=args.served_scale, lambdas=(0.5, 0.8))
    runs = r["runs"]
    out = {"workload": r["config"]["workload"], "resident_points": r["config"]["resident_points"],
           "requests": r["config"]["requests"],
           "results_identical_fifo_vs_batched": r["results_identical_fifo_vs_batched"],
           "saturation_requests_per_s": {m: runs["saturation"][m]["requests_per_s"]
                                         for m in ("fifo", "batched")},
           "saturation_speedup_batched_over_fifo": r["saturation_speedup_batched_over_fifo"]}
    for lam in (0.5, 0.8):
        row = runs[f"lambda_{lam}"]
        out[f"lambda_{lam}"] = {m: {"latency_ms": row[m]["latency_ms"],
                                    "knn_latency_ms": row[m]["knn_latency_ms"],
                                    "requests_per_s": row[m]["requests_per_s"]}
                                for m in ("fifo", "batched")}
    return out


def clustered_leg(args):
    """The 7D clustered workload (10M points in 100 Gaussian blobs, 100
    Insert_L of 100K, one Erase_L of 1M, kNN_L k = 10 for every live point):
    throughput, the traversal's roofline, the self-match property and rows
    sampled against brute force over the live set."""
    import oracle

    a = argparse.Namespace(**vars(args))
    a.workload = "clustered7d_10m"
    a.scale = 1.0
    a.steps = args.clustered_steps
    a.warmup = 1
    r, w, (q, gi, gd) = gpu_bench(a)
    ins = [op for op in w.ops if op.kind == "insert"]
    er = set(int(x) for op in w.ops if op.kind == "erase" for x in op.ids)
    allp = np.concatenate([op.pts for op in ins])
    alli = np.concatenate([op.ids for op in ins])
    live = np.array([int(i) not in er for i in alli])
    qop = [op for op in w.ops if op.kind == "knn"][0]
    sel = np.sort(np.random.default_rng(7).choice(qop.n, size=24, replace=False))
    oi, od = oracle.bruteforce_knn(allp[live], alli[live], qop.pts[sel], qop.k)
    g_i = gi.cpu().numpy().view(np.uint32)[sel]
    g_d = gd.cpu().numpy()[sel]
    keep = ("value", "unit", "ms_per_step", "steps", "config", "knn_queries_per_s",
            "insert_pts_per_s", "erase_pts_per_s", "phase_ms_per_step", "knn_work_per_query",
            "final_levels", "buffer_points", "self_match_all_queries",
            "self_match_own_id_fraction", "insert_roofline")
    out = {kk: r[kk] for kk in keep}
    rf = r["roofline"]
    out["roofline"] = {kk: rf[kk] for kk in ("kernel", "bound", "achieved", "peak", "unit", "frac",
                                             "algorithmic_bytes_per_launch", "avg_launch_ms")}
    out["bruteforce_rows"] = {"rows": len(sel), "equal": bool(
        np.array_equal(g_i, oi) and np.array_equal(g_d.view(np.uint32), od.view(np.uint32)))}
    return out


def host_cpu_model() -> str:
    """The host CPU's model name (what lscpu reports), from /proc/cpuinfo."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def cpu_baseline(w, gpu_out, n_sample: int, n_sample_par: int):
    """The oracle on the host cores.  The updates (every Insert_L and the
    Erase_L of the step, at full size) run serially: the oracle's update code
    is serial.  kNN_L runs (i) serially on a sample of the queries and (ii)
    with the queries spread over all host threads (OpenMP) on a larger
    sample; the kNN time is scaled from the sample to all queries.  `value`
    uses the all-cores kNN time."""
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
    rng = np.random.default_rng(123)
    sel = np.sort(rng.choice(nq, size=min(n_sample, nq), replace=False))
    t0 = time.perf_counter()
    oi, od, cnt = o.knn(qop.pts[sel], qop.k, counters=True)
    t_knn = time.perf_counter() - t0
    sel_p = np.sort(rng.choice(nq, size=min(n_sample_par, nq), replace=False))
    t0 = time.perf_counter()
    pi, pd, threads, _ = o.knn_parallel(qop.pts[sel_p], qop.k)
    t_knn_p = time.perf_counter() - t0
    # parity on both samples at full size
    q, gi, gd = gpu_out
    g_ids = gi.cpu().numpy().view(np.uint32)
    g_d2 = gd.cpu().numpy().view(np.uint32)
    ids_equal = bool(np.array_equal(g_ids[sel], oi) and np.array_equal(g_ids[sel_p], pi))
    d2_equal = bool(np.array_equal(g_d2[sel], od.view(np.uint32)) and
                    np.array_equal(g_d2[sel_p], pd.view(np.uint32)))
    o.close()
    t_par = t_ins + t_er + t_knn_p * nq / len(sel_p)
    t_ser = t_ins + t_er + t_knn * nq / len(sel)
    unit = "ops/s (inserted + erased points + kNN queries per second)"
    return {
        "value": (n_ins + n_er + nq) / t_par,
        "unit": unit,
        "cores": threads,
        "kind": "oracle",
        "sample": (f"oracle at full size: all {n_ins} inserted points and {n_er} erases run "
                   f"serially (its update code is serial); kNN_L on {len(sel_p)} of {nq} "
                   f"queries over {threads} host threads (OpenMP over queries), time scaled "
                   f"to all queries"),
        "insert_pts_per_s": n_ins / t_ins,
        "erase_pts_per_s": n_er / t_er,
        "knn_queries_per_s": len(sel_p) / t_knn_p,
        "serial": {"value": (n_ins + n_er + nq) / t_ser, "unit": unit, "cores": 1,
                   "knn_queries_per_s": len(sel) / t_knn, "knn_sample": len(sel)},
        "seconds": t_ins + t_er + t_knn + t_knn_p,
        "host": {"nproc": os.cpu_count(), "threads_used": threads, "cpu": host_cpu_model(),
                 "omp_num_threads": os.environ.get("OMP_NUM_THREADS")},
        "oracle_work_per_query": {"node_visits": cnt["node_visits"] / len(sel),
                                  "dist_evals": cnt["dist_evals"] / len(sel)},
        "gpu_matches_oracle_on_sample": {"ids": ids_equal, "d2_bitwise": d2_equal},
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="uniform3d_10m")
    ap.add_argument("--scale", type=float, default=1.0)
    ap.add_argument("--knn-kernel", type=int, default=2, choices=[0, 1, 2],
                    help="0: one lane per query, 1: one wavefront per group of 64 or 128 queries, "
                         "2: chosen per launch from the query density")
    ap.add_argument("--cpu-sample", type=int, default=200_000,
                    help="queries the serial CPU oracle answers for the baseline (0: skip)")
    ap.add_argument("--cpu-sample-par", type=int, default=1_000_000,
                    help="queries the all-cores CPU oracle answers for the baseline")
    ap.add_argument("--form", default="plain", choices=["plain", "batched", "served", "mixed"])
    ap.add_argument("--mixed-workload", default="mixed2d_10m",
                    choices=["mixed2d_10m", "mixed7d_10m"])
    ap.add_argument("--mixed-scale", type=float, default=0.1,
                    help="scale of the mixed-operations leg of the plain form (0: skip)")
    ap.add_argument("--extra", type=int, default=1,
                    help="1: the plain form also runs the served leg (mixed-load p50/p99) "
                         "and the 7D clustered workload; 0: the 3D step only")
    ap.add_argument("--served-scale", type=float, default=0.2,
                    help="scale of the served leg of the plain form (0: skip)")
    ap.add_argument("--clustered-steps", type=int, default=2,
                    help="timed steps of the 7D clustered leg of the plain form (0: skip)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="run a plain device copy of this size first (counter scaling)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)
    if args.form == "batched":
        print(json.dumps(batched_bench(args)), flush=True)
        return
    if args.form == "served":
        print(json.dumps(served_bench(args)), flush=True)
        return
    if args.form == "mixed":
        print(json.dumps(mixed_bench(args)), flush=True)
        return
    res, w, gpu_out = gpu_bench(args)
    if args.cpu_sample > 0:
        res["cpu_baseline"] = cpu_baseline(w, gpu_out, args.cpu_sample, args.cpu_sample_par)
    else:
        res["cpu_baseline"] = None
    if args.extra:
        if args.clustered_steps > 0:
            print("bench: 7D clustered workload", file=sys.stderr, flush=True)
            res["clustered7d_10m"] = clustered_leg(args)
        if args.served_scale > 0:
            print("bench: served leg", file=sys.stderr, flush=True)
            res["served_mixed_load"] = served_leg(args)
        if args.mixed_scale > 0:
            print("bench: mixed-operations leg", file=sys.stderr, flush=True)
            m = mixed_bench(args, "mixed2d_10m", args.mixed_scale)
            res["mixed_operations"] = {kk: m[kk] for kk in (
                "config", "best_total", "speedup_bdl_over_rebuild_all",
                "speedup_bdl_over_no_rebuild", "bruteforce_rows")}
            res["mixed_operations"]["total_ms"] = {kk: v["total_ms"]
                                                   for kk, v in m["structures"].items()}
            res["mixed_operations"]["knn_rows_equal"] = all(
                v["knn_rows_equal_to_bdl"] is not False for v in m["structures"].values())
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
