"""Autotuner over the paper's design space and the kernel variants.

Three searches, all timed on the device by the library itself:

* :func:`sweep_plans` -- every (operation order, stream map) of the SpMV DAG
  (the design space of Sec. III-B/C, enumerated by the library), timed with
  the paper's benchmark protocol (Sec. III-C3): a measurement repeats the
  program until t_measure = 0.01 s has elapsed and records time / samples.
  Plan objects are re-ordered in place (``spmv_plan_reorder``), so the share
  is uploaded once per replica; samples rotate over cold replicas.
* :func:`tune_kernel` -- the product kernel variant (stream CSR in packed
  tiles: window chunk, load width, summing lanes; sliced ELL: entries per
  batch of loads; vector CSR: lanes per row, rows per lane group; for y_R
  also column slabs), timed with HIP events around back-to-back launches
  over cold replicas.
* :func:`tune_batch_kernels` -- the kernel variants of a batch's shares
  (window, load width, summing lanes of y_L and y_R, y_R in packed tiles or
  column slabs), timed on the batch's grouped device phase over a sample
  of its shares.
* :func:`tune_batch` -- the options of a batch of shares (stream launches
  or one graph, copy streams, pipeline chunks, persistent blocks per CU,
  XCD affinity), timed over whole batches.

Results can be appended to a JSONL cache keyed by the matrix digest, so an
interrupted sweep resumes where it stopped.
"""
from __future__ import annotations

import hashlib
import json
import math
import os

import numpy as np

from . import (SPMV_OP_YL, SPMV_OP_YR, SpmvError, spmv_batch_create, spmv_batch_destroy, spmv_batch_exec,
               spmv_op_launch, spmv_plan_create, spmv_plan_destroy,
               spmv_plan_get_i32, spmv_plan_inbox, spmv_plan_info, spmv_plan_reorder,
               spmv_plan_space_count, spmv_plan_space_get, spmv_plan_time, SPMV_I32_HALO_COLS)

MALL_BYTES = 256 << 20


def matrix_digest(A, nranks: int, rank: int) -> str:
    h = hashlib.blake2b(digest_size=16)
    for a in (A.row_ptr, A.col_idx, A.val):
        h.update(np.ascontiguousarray(a).view(np.uint8))
    h.update(f"{A.n_rows}:{nranks}:{rank}".encode())
    return h.hexdigest()


def _load_cache(path, key):
    done = {}
    if path and os.path.exists(path):
        with open(path) as f:
            for line in f:
                try:
                    d = json.loads(line)
                except json.JSONDecodeError:
                    continue
                if d.get("key") == key:
                    done[d["index"]] = d
    return done


def sweep_plans(A, nranks: int, rank: int, x: np.ndarray, n_streams: int = 2,
                tune: dict | None = None, t_measure: float = 0.01, n_measure: int = 1,
                indices=None, cache_path: str | None = None, replicas: int = 1, log=None):
    """Time every plan of the design space on rank ``rank``'s share.

    With replicas > 1 the share is uploaded that many times and the samples
    of a measurement rotate over the copies (each one re-ordered to the
    candidate plan), so plans are ranked with the matrix streamed from HBM
    as in a cold run.  Returns a list of dicts {index, times (s), t (median
    s)} in index order.
    """
    import torch
    n_plans = spmv_plan_space_count(nranks, n_streams)
    idx = list(range(n_plans)) if indices is None else list(indices)
    key = (f"{matrix_digest(A, nranks, rank)}:{n_streams}:{replicas}:"
           f"{json.dumps(tune or {}, sort_keys=True)}")
    done = _load_cache(cache_path, key)
    ops0, smap0 = spmv_plan_space_get(nranks, n_streams, 0)
    plans = [spmv_plan_create(A, nranks, rank, ops0, smap0, n_streams, tune)
             for _ in range(max(1, replicas))]
    out = []
    try:
        info = spmv_plan_info(plans[0])
        lo, n = info["lo"], info["n_loc"]
        halo = spmv_plan_get_i32(plans[0], SPMV_I32_HALO_COLS).astype(np.int64)
        xs, ys = [], []
        for p in plans:
            spmv_plan_inbox(p)[:] = x[halo]
            xs.append(torch.from_numpy(np.ascontiguousarray(x[lo:lo + n])).cuda())
            ys.append(torch.empty(n, dtype=torch.float64, device="cuda"))
        stream = torch.cuda.current_stream()
        torch.cuda.synchronize()
        # warm-up on both sides of a device-wide synchronisation: the first
        # execs of a process ran their send and receive copies one after the
        # other (the power-law share's step: 695 us instead of 441 us) until
        # a device synchronisation followed them, and the first measurement
        # after it is slow once more
        spmv_plan_time(plans, xs, ys, stream, t_measure, 1)
        torch.cuda.synchronize()
        spmv_plan_time(plans, xs, ys, stream, t_measure, 2)
        fh = open(cache_path, "a") if cache_path else None
        try:
            for j, i in enumerate(idx):
                if i in done:
                    out.append(done[i])
                    continue
                ops, smap = spmv_plan_space_get(nranks, n_streams, i)
                for p in plans:
                    spmv_plan_reorder(p, ops, smap, n_streams)
                t = spmv_plan_time(plans, xs, ys, stream, t_measure, n_measure)
                d = {"key": key, "index": i, "times": t.tolist(), "t": float(np.median(t))}
                out.append(d)
                if fh:
                    fh.write(json.dumps(d) + "\n")
                    fh.flush()
                if log and j % 250 == 0:
                    log(f"plan {j}/{len(idx)}: {d['t'] * 1e6:.1f} us")
        finally:
            if fh:
                fh.close()
    finally:
        for p in plans:
            spmv_plan_destroy(p)
    return out


def best_plans(results, k: int = 1):
    return sorted(results, key=lambda d: d["t"])[:k]


def sweep_summary(results) -> dict:
    t = np.array([d["t"] for d in results])
    i_best = int(np.argmin(t))
    i_worst = int(np.argmax(t))
    pct = (0, 1, 5, 10, 25, 50, 75, 90, 95, 99, 100)
    return {"n_plans": int(t.size), "fastest_us": round(float(t[i_best]) * 1e6, 3),
            "curve_us": {str(q): round(float(np.percentile(t, q)) * 1e6, 2) for q in pct},
            "slowest_us": round(float(t[i_worst]) * 1e6, 3),
            "median_us": round(float(np.median(t)) * 1e6, 3),
            "slowest_over_fastest": round(float(t[i_worst] / t[i_best]), 3),
            "fastest_index": results[i_best]["index"], "slowest_index": results[i_worst]["index"]}


DEFAULT_CANDIDATES = (
    [{"kernel_local": 2, "form": 3, "chunk_local": c} for c in (8, 16)] +
    [{"kernel_local": 2, "form": 2, "chunk_local": c} for c in (4, 8, 16)] +
    [{"kernel_local": 2, "form": 4, "chunk_local": c, "width": 2} for c in (4, 8, 16)] +
    [{"kernel_local": 2, "form": 1, "chunk_local": c, "width": 2} for c in (4, 8, 16)] +
    [{"kernel_local": 2, "form": 1, "chunk_local": c, "width": 2, "lanes_local": l}
     for c in (4, 8) for l in (1, 2, 4)] +
    [{"kernel_local": 1, "lanes_local": l, "rows_local": r} for l in (8, 32) for r in (4, 8)])


# y_R variants: packed tiles with 1, 2 or 4 summing lanes, the sliced form
# (taken only where its padding stays small), column slabs in tiles of 256 /
# lanes rows (1 or 2 lanes) and in wide tiles (2, 4 or 8 rows per thread,
# windows of 1,024 to 4,096 entries).
DEFAULT_REMOTE_CANDIDATES = (
    [{"kernel_remote": 2, "form": 1, "lanes_remote": l} for l in (1, 2, 4)] +
    [{"kernel_remote": 2, "form": 2}] +
    [{"kernel_remote": 2, "form": 5, "lanes_remote": l, "rows_remote": 1} for l in (1, 2)] +
    [{"kernel_remote": 2, "form": 5, "lanes_remote": 1, "rows_remote": r, "chunk_remote": c}
     for r in (2, 4, 8) for c in (4, 8, 16)])


def tune_kernel(A, nranks: int, rank: int, x: np.ndarray, candidates=DEFAULT_CANDIDATES,
                launches: int = 100, log=None, op: int = SPMV_OP_YL, margin: float = 0.02):
    """Search kernel variants for one product (y_L by default: both CSR
    kernels, stream chunk / width / summing lanes, vector lanes / rows; with
    op = SPMV_OP_YR and DEFAULT_REMOTE_CANDIDATES the forms of y_R) by timing
    back-to-back launches of that op over cold replicas.  The automatic
    choice (an empty tune) is timed too and kept unless a candidate beats it
    by more than ``margin``: rankings inside the timing noise would
    otherwise trade it for a variant no faster.  Returns (best tune dict,
    all results; the automatic choice as {})."""
    import torch
    if op not in (SPMV_OP_YL, SPMV_OP_YR):
        raise ValueError("tune_kernel times y_L or y_R")
    results = []
    stream = torch.cuda.Stream()
    for tune in [{}] + list(candidates):
        p0 = spmv_plan_create(A, nranks, rank, None, None, 2, tune)
        info = spmv_plan_info(p0)
        n = info["n_loc"]
        R = max(1, math.ceil(2 * MALL_BYTES / max(info["device_bytes"] + 16 * n, 1)))
        plans = [p0] + [spmv_plan_create(A, nranks, rank, None, None, 2, tune)
                        for _ in range(R - 1)]
        try:
            lo = info["lo"]
            xs = [torch.from_numpy(np.ascontiguousarray(x[lo:lo + n])).cuda() for _ in plans]
            ys = [torch.empty(n, dtype=torch.float64, device="cuda") for _ in plans]
            torch.cuda.synchronize()
            with torch.cuda.stream(stream):
                for i in range(2 * R):
                    spmv_op_launch(plans[i % R], op, xs[i % R], ys[i % R], stream)
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                for i in range(launches):
                    spmv_op_launch(plans[i % R], op, xs[i % R], ys[i % R], stream)
                e1.record(stream)
            torch.cuda.synchronize()
            us = e0.elapsed_time(e1) * 1e3 / launches
        finally:
            for p in plans:
                spmv_plan_destroy(p)
        results.append({"tune": dict(tune), "us": us})
        if log:
            log(json.dumps(results[-1]))
    best = min(results, key=lambda d: d["us"])
    if best["us"] > results[0]["us"] * (1.0 - margin):
        best = results[0]
    return best["tune"], results


DEFAULT_BATCH_CANDIDATES = (
    [{"use_graph": 2, "copy_streams": 1, "chunks": c} for c in (1, 4, 8, 16)] +
    [{"use_graph": 2, "copy_streams": 2, "chunks": c} for c in (1, 8)] +
    [{"use_graph": 2, "copy_streams": 1, "chunks": 8, "persistent": 1, "blocks_per_cu": b}
     for b in (4, 8)] +
    [{"use_graph": 1, "chunks": c} for c in (1, 8)] +
    [{"use_graph": 2, "copy_streams": 1, "chunks": 8, "xcd_affinity": 2}])

# Kernel variants of a batch's shares: the window (entries per thread) and
# load width every share of a batch has in common, the summing lanes of each
# product, and y_R in packed tiles (form 4: y_L with 16-bit columns where
# they fit) or in column slabs (form 5).
DEFAULT_BATCH_KERNEL_CANDIDATES = (
    [{"kernel_local": 2, "kernel_remote": 2, "chunk_local": c, "chunk_remote": c, "width": w,
      "form": f} for c in (4, 8) for w in (2, 4) for f in (4, 5)] +
    [{"kernel_local": 2, "kernel_remote": 2, "chunk_local": 8, "chunk_remote": 8, "width": 2,
      "form": f, "lanes_local": ll, "lanes_remote": lr}
     for f in (4, 5) for ll, lr in ((1, 1), (2, 2), (1, 4) if f == 4 else (1, 2))])


def tune_batch(plans, xs, ys, candidates=DEFAULT_BATCH_CANDIDATES, reps: int = 3, log=None):
    """Search the batch options (stream launches or one graph, copy streams
    per direction, pipeline chunks, persistent blocks or one block per item,
    blocks per CU, XCD affinity) for a set of
    plans by timing whole batches (halo staging included).  Returns (best
    options, all results); every candidate computes the same bits."""
    import time
    import torch
    stream = torch.cuda.current_stream()
    results = []
    for opts in candidates:
        b = spmv_batch_create(plans, opts)
        try:
            spmv_batch_exec(b, xs, ys, stream)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                spmv_batch_exec(b, xs, ys, stream)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) / reps * 1e3
        finally:
            spmv_batch_destroy(b)
        results.append({"opts": dict(opts), "ms": ms})
        if log:
            log(json.dumps(results[-1]))
    best = min(results, key=lambda d: d["ms"])
    return best["opts"], results


def tune_batch_kernels(make_plan, n_sample: int, xs, ys, candidates=DEFAULT_BATCH_KERNEL_CANDIDATES,
                       reps: int = 3, log=None):
    """Search the shares' kernel variants for a batch: for every candidate
    tune, plans of the first n_sample shares (``make_plan(i, tune)``) are
    built and their grouped device phase (the batch without staging) is
    timed; candidates that cannot form a batch (a form the grouped kernels
    do not run) are recorded as such.  Returns (best tune, all results)."""
    import time
    import torch
    stream = torch.cuda.current_stream()
    results = []
    for tune in candidates:
        plans = []
        try:
            plans = [make_plan(i, tune) for i in range(n_sample)]
            b = spmv_batch_create(plans, {"staging": 1})
        except SpmvError as e:
            for p in plans:
                spmv_plan_destroy(p)
            results.append({"tune": dict(tune), "ms": None, "error": str(e)})
            continue
        try:
            spmv_batch_exec(b, xs[:n_sample], ys[:n_sample], stream)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                spmv_batch_exec(b, xs[:n_sample], ys[:n_sample], stream)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) / reps * 1e3
            infos = [spmv_plan_info(p) for p in plans]
        finally:
            spmv_batch_destroy(b)
            for p in plans:
                spmv_plan_destroy(p)
        results.append({"tune": dict(tune), "ms": ms,
                        "forms": sorted({(i["form_local"], i["form_remote"]) for i in infos}),
                        "lanes": sorted({(i["lanes_local"], i["lanes_remote"]) for i in infos})})
        if log:
            log(json.dumps(results[-1]))
    ok = [d for d in results if d["ms"] is not None]
    if not ok:
        raise SpmvError(-1, "no candidate forms a batch")
    best = min(ok, key=lambda d: d["ms"])
    return best["tune"], results
