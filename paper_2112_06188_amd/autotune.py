"""Launch-shape autotuner for kNN_L on the device at hand.

For each band of k and of query counts it times every candidate shape
(traversal kernel, workgroup size, persistent grid, Hilbert-curve ordering of a
plain call) on the caller's own resident tree with queries the caller
draws, keeps the fastest by median device time, and installs the winners as
the tree's shape table (bdl_set_knn_shapes).  Shapes change speed, never
results; the tuner checks that too, comparing every candidate's output with
the first candidate's, bit for bit.

The table can be saved as JSON and loaded into another tree of the same
dimension on the same kind of device.
"""
from __future__ import annotations

import itertools
import json
import statistics
from typing import Callable, Dict, Iterable, List, Optional, Sequence

KERNELS = (0, 1, 3)      # lane per query, wavefront per 64 queries, wavefront per query
BLOCKS = (64, 128, 256)
PERSISTENT = (0, 1)
SORT = (0, 1)

# bands of the query count: [lo, hi] inclusive, each timed at its upper end
# (at most max_nq)
DEFAULT_NQ_BANDS = ((1, 4096), (4097, 65536), (65537, 1 << 20), ((1 << 20) + 1, 1 << 40))
DEFAULT_K_BANDS = ((1, 1), (2, 5), (6, 10), (11, 64))


def candidates(kernels=KERNELS, blocks=BLOCKS, persistent=PERSISTENT, sort=SORT) -> List[Dict]:
    return [dict(kernel=k, block=b, persistent=p, sort=s)
            for k, b, p, s in itertools.product(kernels, blocks, persistent, sort)]


def _time_call(torch, fn: Callable[[], None], reps: int, stream) -> float:
    """Median device time of fn() in ms over reps runs (after one warm run)."""
    fn()
    times = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        fn()
        b.record(stream)
        b.synchronize()
        times.append(a.elapsed_time(b))
    return statistics.median(times)


def tune(tree, make_queries: Callable[[int], "object"], *,
         k_bands: Sequence = DEFAULT_K_BANDS, nq_bands: Sequence = DEFAULT_NQ_BANDS,
         max_nq: int = 1 << 22, reps: int = 3, cands: Optional[Iterable[Dict]] = None,
         batched: bool = False, install: bool = True, log: Callable[[str], None] = None) -> Dict:
    """Tune the shape table of `tree`.

    make_queries(n) returns n queries as a device tensor [n, dim] float32.
    A band is timed with k = its upper end and nq = min(its upper end,
    max_nq).  batched=True times bdl_knn_batch with one request per call
    (the graph path) instead of bdl_knn.
    Returns {"rows": [...], "timings": [...]} and installs the rows.
    """
    import torch

    cands = list(cands) if cands is not None else candidates()
    stream = tree.stream
    rows, timings = [], []
    saved = list(getattr(tree, "_shapes", []))
    for (klo, khi), (nlo, nhi) in itertools.product(k_bands, nq_bands):
        k = khi
        nq = int(min(nhi, max_nq))
        if nq < nlo:
            continue
        q = make_queries(nq)
        ref = None
        best = None
        for c in cands:
            row = dict(k_lo=klo, k_hi=khi, nq_lo=nlo, nq_hi=nhi, **c)
            tree.set_knn_shapes([row])
            ids = torch.empty((nq, k), dtype=torch.int32, device=q.device)
            d2 = torch.empty((nq, k), dtype=torch.float32, device=q.device)
            if batched:
                fn = lambda: tree.knn_batch([(q, k)], outputs=[(ids, d2)])  # noqa: E731
            else:
                fn = lambda: tree.knn(q, k, ids, d2)  # noqa: E731
            ms = _time_call(torch, fn, reps, stream)
            tree.sync()
            if ref is None:
                ref = (ids.clone(), d2.clone())
            elif not (torch.equal(ids, ref[0]) and
                      torch.equal(d2.view(torch.int32), ref[1].view(torch.int32))):
                raise RuntimeError(f"launch shape {c} changed k-NN results (k={k}, nq={nq})")
            timings.append(dict(row, nq=nq, k=k, ms=ms))
            if best is None or ms < best[0]:
                best = (ms, row)
        if log:
            log(f"k in [{klo},{khi}] nq in [{nlo},{nhi}] (timed k={k} nq={nq}): "
                f"best {best[1]} {best[0]:.3f} ms")
        rows.append(best[1])
    tree.set_knn_shapes(rows if install else saved)
    return {"rows": rows, "timings": timings}


def save(result: Dict, path: str, meta: Optional[Dict] = None) -> None:
    with open(path, "w") as f:
        json.dump({"meta": meta or {}, "rows": result["rows"]}, f, indent=1)


def load(tree, path: str) -> List[Dict]:
    """Install the rows saved by save() into tree; returns them."""
    with open(path) as f:
        rows = json.load(f)["rows"]
    tree.set_knn_shapes(rows)
    return rows
