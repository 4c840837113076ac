#!/usr/bin/env python3
"""Benchmark of the rank-share SpMV on one MI355X.

One step = the whole device work of a rank share with every input (A, x and
the halo the other ranks sent) resident in HBM: Pack, local product y_L,
Unpack and remote product y_R accumulated into y (``spmv_exec_resident``;
where y_R is in column slabs, Pack, y_L and the slab tiles as one grouped
launch, then the slab sums), rotating over cold replicas.  The full program with the exchange emulated
through pinned host memory (``spmv_exec``: the plan's order and streams,
PostSend/PostRecv/Wait*, host-synchronous) is timed beside it and reported
as the PCIe-inclusive rate; it is not the headline value.

The headline share is rank 5 of the 4M-row power-law matrix on 16 ranks
(the whole matrix is generated; the largest single-GPU configuration: its
remote product gathers from a 19 MB halo).  The 3D 7-point 128^3 and 27-point
150^3 shares are measured beside it, the 7-point share with the design-space
stages (plan sweep, design rules and their stability over repeated sweeps,
tree search, fine-grained program, every rank's share), and the paper's own
banded input with its plan sweep and rules.

Cold-cache protocol: a share is uploaded R times (independent device copies
of A, x and y, R * footprint > 2x the 256 MB Infinity Cache) and the steps
rotate over the copies, so each step streams A from HBM.

Printed: one JSON line with the metric ``rank-share SpMV GB/s`` (algorithmic
device bytes of a step / wall time per step), the roofline of the headline
share's dominant kernel (the step's grouped launch, or its largest op;
timed with HIP events on the stream it is launched on) and of its largest
op alone (``op_roofline``: y_R), the staged program's rate, the CPU oracle's rate on a bounded
sample, the 64-share batch and the serving trace.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E peak
MALL_BYTES = 256 << 20         # Infinity Cache
HEADLINE = "powerlaw_4m_p16r5"
EXTRAS = ("laplace3d_128_p4r1", "stencil27_150_p8r3")

# HBM bytes per launch of a kernel from the two rocprofv3 --pmc runs
# (FETCH_SIZE x 1.9994 + WRITE_SIZE x 1.0, factors from the copy probe of
# known size), keyed by workload and kernel variant, with the summary that
# holds them; a variant that is not listed (or a kernel changed since)
# reports null.
MEASURED_TRAFFIC = {
    ("powerlaw_4m_p16r5", "k_csr_slabs<4,2,1>+k_slab_sum"):
        (111_144_633, "profiles/yr_slabs_powerlaw_4m_p16r5.md"),
    ("powerlaw_4m_p16r5", "k_resident<4,2>"):
        (140_957_582, "profiles/resident_grouped_powerlaw_4m_p16r5.md"),
    ("laplace3d_128_p4r1", "k_sell16<1>"):
        (47_998_920, "profiles/sliced16_laplace3d_128_p4r1.md"),
    ("stencil27_150_p8r3", "k_csr_stream<4,2,2,true>"):
        (120_269_255, "profiles/stream_csr_stencil27_150_p8r3.md"),
}

OPS = ("pack", "yL", "unpack", "yR")


def op_code(sp, name: str) -> int:
    return {"pack": sp.SPMV_OP_PACK, "yL": sp.SPMV_OP_YL, "unpack": sp.SPMV_OP_UNPACK,
            "yR": sp.SPMV_OP_YR}[name]


def step_bytes(info: dict) -> dict:
    """Algorithmic device bytes of each GPU step of one exec (unique data
    touched once: index arrays, matrix values, gathered/scattered vectors).
    """
    n, nl, nr = info["n_loc"], info["nnz_local"], info["nnz_remote"]
    h, s, rr = info["n_halo"], info["n_send"], info["n_remote_rows"]
    b = {}
    b["pack"] = 20 * s                                   # idx 4 + x 8 + sendbuf 8
    b["yL"] = 12 * nl + 4 * (n + 1) + 8 * n + 8 * n      # col+val, row_ptr, x, y
    b["unpack"] = 0 if info["fuse_unpack"] else 20 * h   # perm 4 + recv 8 + x_halo 8
    yr = 12 * nr + 4 * (rr + 1) + 4 * rr + 8 * h        # col+val, ptr, row ids, x_halo
    if info["fused_combine"]:
        yr += 16 * rr                                    # y read + write
        b["combine"] = 0
    else:
        yr += 8 * rr                                     # partial sums written
        b["combine"] = 4 * rr + 8 * rr + 16 * rr         # ids, partials, y read+write
    b["yR"] = yr
    b["total"] = sum(v for k, v in b.items())
    b["host_link"] = 8 * (s + h)                         # staged each way
    return b


def launch_bytes(info: dict) -> dict:
    """Algorithmic bytes of one spmv_op_launch of each GPU op (y_R launched
    alone adds into y: its row ids, y read and written).  Where the resident
    step is grouped, also its two launches: Pack, y_L and y_R's slab tiles
    (entries, row pointers, halo), then the slab sums (row ids, y read and
    written); together the bytes of Pack, y_L and y_R."""
    n, nl, nr = info["n_loc"], info["nnz_local"], info["nnz_remote"]
    h, s, rr = info["n_halo"], info["n_send"], info["n_remote_rows"]
    b = {"pack": 20 * s,
         "yL": 12 * nl + 4 * (n + 1) + 16 * n,
         "unpack": 0 if info["fuse_unpack"] else 20 * h,
         "yR": 12 * nr + 4 * (rr + 1) + 4 * rr + 8 * h + 16 * rr if rr else 0}
    if info.get("resident_grouped") == 1:
        b["grouped"] = b["pack"] + b["yL"] + 12 * nr + 4 * (rr + 1) + 8 * h
        b["slab_sums"] = 4 * rr + 16 * rr
    return b


def replicas_for(A, P, r, tune, sp) -> int:
    """Device copies of the share needed to exceed twice the Infinity Cache."""
    p = sp.spmv_plan_create(A, P, r, None, None, 2, {**tune, "flags": sp.SPMV_F_HOST_ONLY})
    try:
        info = sp.spmv_plan_info(p)
    finally:
        sp.spmv_plan_destroy(p)
    n, nl, nr = info["n_loc"], info["nnz_local"], info["nnz_remote"]
    footprint = 12 * (nl + nr) + 4 * n + 24 * (info["n_halo"] + info["n_send"]) + 16 * n
    return max(1, math.ceil(2 * MALL_BYTES / max(footprint, 1)))


def _stream_variant(form, chunk, width, lanes):
    return "k_csr_stream<%d,%d,%d,%s>" % (chunk, width, lanes, "true" if form == 4 else "false")


def kernel_variant(info: dict, side: str = "yL") -> str:
    """Name of the kernel (template instance) that runs one product."""
    loc = side == "yL"
    kern = info["kernel_local" if loc else "kernel_remote"]
    form = info["form_local" if loc else "form_remote"]
    chunk = info["chunk_local" if loc else "chunk_remote"]
    lanes = info["lanes_local" if loc else "lanes_remote"]
    rows = info["rows_local" if loc else "rows_remote"]
    if kern == 2 and form == 3:
        return "k_sell16<%d>" % (chunk // 8)
    if kern == 2 and form == 2:
        return "k_sell<%d>" % chunk
    if kern == 2 and form == 5:
        main = ("k_csr_slabs_wide<%d,%d,%d>" % (chunk, info["width"], rows) if rows > 1
                else "k_csr_slabs<%d,%d,%d>" % (chunk, info["width"], lanes))
        return main + "+k_slab_sum"
    if kern == 2:
        return _stream_variant(form, chunk, info["width"], lanes)
    return "k_csr_vector_buf<%d,%d>" % (lanes, rows)


def time_part(sp, torch, plans, part, xs, ys, launches: int) -> float:
    """Average duration (us) of one of the grouped resident launches, timed
    as time_op times an op."""
    stream = torch.cuda.Stream()
    R = len(plans)
    with torch.cuda.stream(stream):
        for i in range(2 * R):
            sp.spmv_exec_resident_part(plans[i % R], part, xs[i % R], ys[i % R], stream)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for i in range(launches):
            sp.spmv_exec_resident_part(plans[i % R], part, xs[i % R], ys[i % R], stream)
        e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) * 1e3 / launches


def grouped_variant(info: dict) -> str:
    return "k_resident<%d,%d>" % (info["chunk_local"], info["width"])


def time_op(sp, torch, plans, op, xs, ys, launches: int) -> float:
    """Average duration (us) of one GPU op of the plan: HIP events bracket
    `launches` back-to-back launches on the stream they are issued to,
    rotating over the cold replicas, so launch gaps are hidden behind the
    queued kernels."""
    stream = torch.cuda.Stream()
    R = len(plans)
    with torch.cuda.stream(stream):
        for i in range(2 * R):
            sp.spmv_op_launch(plans[i % R], op, xs[i % R], ys[i % R], stream)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for i in range(launches):
            sp.spmv_op_launch(plans[i % R], op, xs[i % R], ys[i % R], stream)
        e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) * 1e3 / launches


_T_START = time.perf_counter()


def progress(msg: str) -> None:
    """One line on stderr as each section of the run finishes (stdout holds
    only the JSON result)."""
    print(f"[bench {time.perf_counter() - _T_START:7.1f} s] {msg}", file=sys.stderr, flush=True)


def probe_ceiling(sp, torch, nbytes: int, launches: int = 200) -> dict:
    """Achievable read bandwidth at a given size: the read probe over cold
    buffers of `nbytes` (rotated past twice the MALL), best of a few grid
    sizes."""
    nbytes = max(16, nbytes // 16 * 16)
    K = max(2, math.ceil(2 * MALL_BYTES / nbytes))
    bufs = [torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").fill_(1.0)
            for _ in range(K)]
    part = torch.empty(1 << 16, dtype=torch.float64, device="cuda")
    stream = torch.cuda.Stream()
    best = None
    for blocks in (1024, 2048, 4096, 8192):
        with torch.cuda.stream(stream):
            for i in range(2 * K):
                sp.spmv_hbm_probe(0, bufs[i % K], part, nbytes, blocks, stream)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for i in range(launches):
                sp.spmv_hbm_probe(0, bufs[i % K], part, nbytes, blocks, stream)
            e1.record(stream)
        torch.cuda.synchronize()
        us = e0.elapsed_time(e1) * 1e3 / launches
        if best is None or us < best[1]:
            best = (blocks, us)
    del bufs
    gbs = nbytes / (best[1] * 1e-6) / 1e9
    return {"bytes": nbytes, "blocks": best[0], "us": round(best[1], 3),
            "read_gbs": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4)}


def gather_ceiling(sp, torch, n_gathers: int, window_doubles: int, launches: int = 200) -> dict:
    """What the L2 and the MALL serve of random 8-byte gathers: the gather
    probe making about n_gathers loads, each block inside its XCD's window
    of window_doubles (the column-slab pattern; per_xcd) and over all 8
    windows at once (a halo larger than the L2; whole)."""
    per_block = sp.spmv_gathers_per_probe_block()
    blocks = max(8, -(-n_gathers // per_block))
    src = torch.ones(8 * window_doubles, dtype=torch.float64, device="cuda")
    part = torch.empty(blocks, dtype=torch.float64, device="cuda")
    stream = torch.cuda.Stream()
    out = {"gathers": blocks * per_block, "window_bytes": 8 * window_doubles}
    for name, mode in (("per_xcd_us", 2), ("whole_us", 3)):
        with torch.cuda.stream(stream):
            for _ in range(20):
                sp.spmv_hbm_probe(mode, src, part, src.numel() * 8, blocks, stream)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(launches):
                sp.spmv_hbm_probe(mode, src, part, src.numel() * 8, blocks, stream)
            e1.record(stream)
        torch.cuda.synchronize()
        out[name] = round(e0.elapsed_time(e1) * 1e3 / launches, 3)
    return out


def host_cpu() -> dict:
    """The host's CPU model and logical core count."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": os.cpu_count()}


def _share_rows(A, P, r):
    import oracle
    lo_all = oracle.row_blocks(A.n_rows, P)
    lo, hi = int(lo_all[r]), int(lo_all[r + 1])
    return lo, hi, np.ascontiguousarray(A.row_ptr[lo:hi + 1])


def _timed_repeats(fn, budget_s: float):
    fn()                                                      # warm-up
    times = []
    t_start = time.perf_counter()
    while len(times) < 5 or time.perf_counter() - t_start < budget_s:
        t0 = time.perf_counter()
        fn()
        times.append(time.perf_counter() - t0)
    return float(np.median(times)), len(times), time.perf_counter() - t_start


def cpu_baseline(A, P, r, x, bytes_per_step: float, dynamic: bool,
                 budget_s: float = 12.0) -> dict:
    """The oracle (Dot2 over every owned row, OpenMP on all host threads)
    timed on the host: full rank-share products repeated for about budget_s
    seconds of CPU work, median."""
    import oracle
    oracle.build(force=False)
    lo, hi, rp = _share_rows(A, P, r)
    t, k, wall = _timed_repeats(lambda: oracle.spmv_dot2(rp, A.col_idx, A.val, x, dynamic),
                                budget_s)
    return {"value": round(bytes_per_step / t / 1e9, 3), "unit": "GB/s",
            "cores": oracle.num_threads(), "kind": "oracle", **host_cpu(),
            "schedule": "dynamic,1024" if dynamic else "static",
            "sample": f"{k} full rank-share products (Dot2, all {hi - lo} owned rows) "
                      f"in {wall:.1f} s, median {t * 1e3:.3f} ms each"}


def cpu_plain(A, P, r, x, bytes_per_step: float, dynamic: bool, budget_s: float = 6.0) -> dict:
    """The plain FP64 CSR product of the same rows (one multiply and add per
    entry, OpenMP over rows on all host threads): the ordinary CPU way to
    compute this share, beside the oracle."""
    import oracle
    lo, hi, rp = _share_rows(A, P, r)
    t, k, wall = _timed_repeats(lambda: oracle.spmv_plain(rp, A.col_idx, A.val, x, dynamic),
                                budget_s)
    return {"value": round(bytes_per_step / t / 1e9, 3), "unit": "GB/s",
            "cores": oracle.num_threads(), "kind": "plain CSR loop, OpenMP", **host_cpu(),
            "schedule": "dynamic,1024" if dynamic else "static",
            "gflops": round(2.0 * int(A.row_ptr[hi] - A.row_ptr[lo]) / t / 1e9, 3),
            "sample": f"{k} full rank-share products in {wall:.1f} s, median "
                      f"{t * 1e3:.3f} ms each"}


def batched_section(sp, torch, gen, n_shares: int, reps: int) -> dict:
    """64 power-law rank shares (4M rows, 16 ranks, rank 5, one seed each) in
    one batch: the shares' kernel variants searched on the batch's grouped
    device phase over a sample of 8 shares, the batch options (copy streams,
    pipeline chunks, grid, graph) searched over whole batches with the halo
    staged, then the chosen batch timed against the same shares run one
    spmv_exec after another."""
    from paper_2203_02530_amd import tune as tuner
    t_gen = time.perf_counter()
    shares, xs, ys = [], [], []
    for i in range(n_shares):
        d = gen.power_law_share(4_000_000, 16, 5, seed=4000 + i)
        x = gen.x_normal(d["n_global"], 4100 + i)
        shares.append((d, x))
    t_gen = time.perf_counter() - t_gen

    def make_plan(i, tune):
        d, x = shares[i]
        p = sp.spmv_plan_create_local(d["local"], d["n_global"], 16, 5, d["send_idx"],
                                      d["send_off"], tune=tune)
        halo = sp.spmv_plan_get_i32(p, sp.SPMV_I32_HALO_COLS).astype(np.int64)
        sp.spmv_plan_inbox(p)[:] = x[halo]
        return p
    for d, x in shares:
        lo, n = d["lo"], d["local"].n_rows
        xs.append(torch.from_numpy(np.ascontiguousarray(x[lo:lo + n])).cuda())
        ys.append(torch.empty(n, dtype=torch.float64, device="cuda"))
    stream = torch.cuda.current_stream()
    out = {"workload": f"{n_shares} power-law rank shares: 4M rows, lognormal(16, 1.2) row "
                       f"lengths, 16 ranks, rank 5, seeds 4000..{4000 + n_shares - 1}"}
    t0 = time.perf_counter()
    kbest, kres = tuner.tune_batch_kernels(make_plan, min(8, n_shares), xs, ys, reps=3)
    t_ktune = time.perf_counter() - t0
    plans = []
    try:
        plans = [make_plan(i, kbest) for i in range(n_shares)]

        def timed(fn, k):
            fn()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(k):
                fn()
            torch.cuda.synchronize()
            return (time.perf_counter() - t0) / k

        t0 = time.perf_counter()
        tuned, tune_res = tuner.tune_batch(plans, xs, ys, reps=2)
        t_btune = time.perf_counter() - t0
        bt = sp.spmv_batch_create(plans, tuned)
        dev = sp.spmv_batch_create(plans, {"staging": 1,
                                           "persistent": tuned.get("persistent", 0),
                                           "blocks_per_cu": tuned.get("blocks_per_cu", 0)})
        try:
            finfo = sp.spmv_batch_info(bt)
            t_batch = timed(lambda: sp.spmv_batch_exec(bt, xs, ys, stream), reps)
            t_dev = timed(lambda: sp.spmv_batch_exec(dev, xs, ys, stream), reps * 4)

            def sequential():
                for p, x_, y_ in zip(plans, xs, ys):
                    sp.spmv_exec(p, x_, y_, stream)
            t_seq = timed(sequential, max(1, reps // 2))
        finally:
            sp.spmv_batch_destroy(bt)
            sp.spmv_batch_destroy(dev)
        infos = [sp.spmv_plan_info(p) for p in plans]
        variants = {}
        for inf in infos:
            key = f"y_L {kernel_variant(inf, 'yL')}, y_R {kernel_variant(inf, 'yR')}"
            variants[key] = variants.get(key, 0) + 1
        B = finfo["device_bytes"]
        out.update({
            "shares": n_shares, "work_items": finfo["n_items"], "grid": finfo["n_blocks"],
            "chunks": finfo["n_chunks"], "persistent": finfo["persistent"],
            "ms_per_batch": round(t_batch * 1e3, 3),
            "ms_per_batch_device_phase": round(t_dev * 1e3, 3),
            "ms_sequential_execs": round(t_seq * 1e3, 3),
            "speedup_vs_sequential": round(t_seq / t_batch, 3),
            "share_variants": variants,
            "kernel_autotune": {"sample_shares": min(8, n_shares), "wall_s": round(t_ktune, 1),
                                "best": kbest,
                                "candidates": [{"tune": d["tune"],
                                                "ms": None if d["ms"] is None else round(d["ms"], 3),
                                                **({"forms": d["forms"]} if "forms" in d else {})}
                                               for d in kres]},
            "batch_autotune": {"opts": tuned, "wall_s": round(t_btune, 1),
                               "candidates": [{"opts": d["opts"], "ms": round(d["ms"], 3)}
                                              for d in tune_res]},
            "shares_per_s": round(n_shares / t_batch, 1),
            "device_bytes_per_batch": B,
            "device_phase_gbs": round(B / t_dev / 1e9, 1),
            "device_phase_frac_of_peak": round(B / t_dev / 1e9 / HBM_PEAK_GBS, 4),
            "host_link_bytes_per_batch": finfo["host_link_bytes"],
            "host_link_gbs": round(finfo["host_link_bytes"] / t_batch / 1e9, 2),
            "input_build_s": round(t_gen, 1)})
    finally:
        for p in plans:
            sp.spmv_plan_destroy(p)
    return out


# the shares' kernel variant the batch autotuner picks on the power-law
# shares (y_R in column slabs, windows of 1,024 entries, 2-wide loads)
BATCH_TUNE = {"kernel_local": 2, "kernel_remote": 2, "chunk_local": 4, "chunk_remote": 4,
              "width": 2, "form": 5}


def batch_device_only(sp, torch, gen, n_shares: int, reps: int, opts: dict) -> dict:
    """The device phase of the power-law batch alone (grouped kernels, no
    staging), repeated: what a profiler run of the batch traces."""
    plans, xs, ys = [], [], []
    try:
        for i in range(n_shares):
            d = gen.power_law_share(4_000_000, 16, 5, seed=4000 + i)
            x = gen.x_normal(d["n_global"], 4100 + i)
            p = sp.spmv_plan_create_local(d["local"], d["n_global"], 16, 5, d["send_idx"],
                                          d["send_off"], tune=BATCH_TUNE)
            plans.append(p)
            halo = sp.spmv_plan_get_i32(p, sp.SPMV_I32_HALO_COLS).astype(np.int64)
            sp.spmv_plan_inbox(p)[:] = x[halo]
            xs.append(torch.from_numpy(np.ascontiguousarray(x[d["lo"]:d["lo"] + d["local"].n_rows]))
                      .cuda())
            ys.append(torch.empty(d["local"].n_rows, dtype=torch.float64, device="cuda"))
        progress("batch device phase")
        b = sp.spmv_batch_create(plans, {**opts, "staging": 1})
        try:
            info = sp.spmv_batch_info(b)
            stream = torch.cuda.current_stream()
            sp.spmv_batch_exec(b, xs, ys, stream)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                sp.spmv_batch_exec(b, xs, ys, stream)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) / reps * 1e3
        finally:
            sp.spmv_batch_destroy(b)
    finally:
        for p in plans:
            sp.spmv_plan_destroy(p)
    return {"batch_device_only": True, "shares": n_shares, "tune": BATCH_TUNE, "reps": reps,
            "opts": opts, "ms": round(ms, 3), "chunks": info["n_chunks"],
            "persistent": info["persistent"], "grid": info["n_blocks"],
            "device_bytes": info["device_bytes"],
            "gbs": round(info["device_bytes"] / (ms * 1e-3) / 1e9, 1)}


def serving_section(sp, torch, gen, n_req: int, rate: float, n_mats: int) -> dict:
    """Continuous-batching server vs the plain per-call path on one Poisson
    trace over a pool of resident banded-random matrices."""
    rng = np.random.default_rng(5000)
    sizes = np.rint(10 ** rng.uniform(3, 6, n_mats)).astype(np.int64)
    t_gen = time.perf_counter()
    pool = [gen.banded_random(int(sizes[i]), 5, 27, 2000, seed=5000 + i) for i in range(n_mats)]
    t_gen = time.perf_counter() - t_gen
    tr = np.random.default_rng(5200)
    arrival = np.cumsum(tr.exponential(1.0 / rate, n_req))
    arrival -= arrival[0]
    mat = tr.integers(0, n_mats, n_req).astype(np.int32)
    # fresh x per request: distinct windows of one pinned N(0,1) pool; y:
    # rotating windows of a pinned arena (results are not inspected here)
    xpool = torch.from_numpy(np.random.default_rng(5300).standard_normal(16 << 20)).pin_memory()
    yarena = torch.empty(64 << 20, dtype=torch.float64).pin_memory()
    xb, yb = xpool.data_ptr(), yarena.data_ptr()
    xs, ys, yoff = [], [], 0
    for i in range(n_req):
        n = int(sizes[mat[i]])
        xs.append(xb + 8 * ((i * 1_000_003) % (xpool.numel() - n)))
        if yoff + n > yarena.numel():
            yoff = 0
        ys.append(yb + 8 * yoff)
        yoff += n
    out = {"workload": f"{n_req} requests, Poisson {rate:.0f}/s, pool of {n_mats} resident "
                       "banded-random matrices (rows 1e3..1e6 log-uniform, 5..27 nnz/row, "
                       "half-bandwidth 2000), 64 GiB budget",
           "pool_rows": int(sizes.sum()), "pool_nnz": int(sum(A.nnz for A in pool)),
           "input_build_s": round(t_gen, 1)}
    # the Poisson trace at the target rate, the same arrivals three times
    # denser (where requests start to overlap on the device), then all
    # requests arriving at once (the servers' saturated throughput)
    burst = np.zeros(n_req)
    for label, arr in (("", arrival), ("x3_rate_", arrival / 3.0), ("saturated_", burst)):
        for name, mode in (("batched", 0), ("plain", 1)):
            srv = sp.spmv_server_create({"mode": mode})
            try:
                for A in pool:
                    sp.spmv_server_add_matrix(srv, A)
                sp.spmv_server_start(srv)
                lat, wall = sp.spmv_server_run_trace(srv, mat, arr, xs, ys)
                st = sp.spmv_server_stats(srv)
            finally:
                sp.spmv_server_destroy(srv)
            out[label + name] = {"req_per_s": round(n_req / wall, 1),
                                 "p50_us": round(float(np.percentile(lat, 50)) * 1e6, 1),
                                 "p99_us": round(float(np.percentile(lat, 99)) * 1e6, 1),
                                 "mean_us": round(float(lat.mean()) * 1e6, 1),
                                 "mean_batch": round(st["mean_batch"], 2),
                                 "batches": st["batches"], "peak_inflight": st["peak_inflight"],
                                 "resident_gb": round(st["resident_bytes"] / 1e9, 3)}
    out["p99_plain_over_batched"] = round(out["plain"]["p99_us"] / out["batched"]["p99_us"], 3)
    out["x3_rate_p99_plain_over_batched"] = round(
        out["x3_rate_plain"]["p99_us"] / out["x3_rate_batched"]["p99_us"], 3)
    out["saturated_throughput_batched_over_plain"] = round(
        out["saturated_batched"]["req_per_s"] / out["saturated_plain"]["req_per_s"], 3)
    return out


def rules_section(sp, torch, A, P, r, x, sweep_res, replicas, ktune, live=True) -> dict:
    """Design rules from the exhaustive sweep (Sec. IV), the Table V
    experiment on those times (classes and tree from tree-search subsets,
    accuracy over the whole space), and one live tree search on the device."""
    from paper_2203_02530_amd import rules
    t_all = np.empty(len(sweep_res))
    for d in sweep_res:
        t_all[d["index"]] = d["t"]
    space = rules.plan_space(P, 2)
    dr = rules.design_rules(space, t_all)
    y = dr["labels"]["labels"]
    classes = [{"class": int(c), "n": int((y == c).sum()),
                "us": [round(float(t_all[y == c].min()) * 1e6, 2),
                       round(float(t_all[y == c].max()) * 1e6, 2)]} for c in np.unique(y)]
    top = {}
    for rs in dr["rules"]:
        top.setdefault(rs["class"], [])
        if len(top[rs["class"]]) < 3:
            top[rs["class"]].append({"samples": rs["samples"], "rules": rs["text"]})
    table_v = {}
    for it in (50, 100, 200, 400, 0):
        res = sp.spmv_mcts_run_table(P, t_all, iterations=it, seed=1)
        acc = rules.class_accuracy(space, t_all, res["index"])
        table_v[str(it or len(space))] = round(acc["accuracy"], 3)
    out = {"n_classes": len(classes), "classes": classes, "leaves": dr["mln"],
           "depth": int(dr["tree"].get_depth()) if dr["tree"] is not None else 0,
           "n_features": len(dr["names"]), "rules_top3": top, "table_v_accuracy": table_v}
    if not live:
        return out
    # live search: rollouts timed on the device over cold replicas
    plans = [sp.spmv_plan_create(A, P, r, None, None, 2, ktune) for _ in range(replicas)]
    try:
        info = sp.spmv_plan_info(plans[0])
        lo, n = info["lo"], info["n_loc"]
        halo = sp.spmv_plan_get_i32(plans[0], sp.SPMV_I32_HALO_COLS).astype(np.int64)
        xs, ys = [], []
        for p in plans:
            sp.spmv_plan_inbox(p)[:] = x[halo]
            xs.append(torch.from_numpy(np.ascontiguousarray(x[lo:lo + n])).cuda())
            ys.append(torch.empty(n, dtype=torch.float64, device="cuda"))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        found = sp.spmv_mcts_run(plans, xs, ys, torch.cuda.current_stream(), iterations=200,
                                 seed=2)
        wall = time.perf_counter() - t0
    finally:
        for p in plans:
            sp.spmv_plan_destroy(p)
    best_live = int(found["index"][int(np.argmin(found["time"]))])
    return {**out,
            "live_search": {"iterations": int(found["index"].size), "wall_s": round(wall, 2),
                            "best_us": round(float(found["time"].min()) * 1e6, 2),
                            "best_index": best_live,
                            "best_class_in_sweep": int(y[best_live]),
                            "sweep_fastest_us": round(float(t_all.min()) * 1e6, 2)}}


def fine_section(sp, torch, A, P, r, x, replicas, ktune, coarse_best, iterations=400) -> dict:
    """The fine-grained program (per-peer Pack / copies / waits, Sec. III-A):
    a device-timed tree search over its DAG, then the best fine program and
    the best coarse plan re-measured side by side on the same cold replicas."""
    plans = [sp.spmv_plan_create(A, P, r, None, None, 2, ktune) for _ in range(replicas)]
    try:
        info = sp.spmv_plan_info(plans[0])
        lo, n = info["lo"], info["n_loc"]
        halo = sp.spmv_plan_get_i32(plans[0], sp.SPMV_I32_HALO_COLS).astype(np.int64)
        xs, ys = [], []
        for p in plans:
            sp.spmv_plan_inbox(p)[:] = x[halo]
            xs.append(torch.from_numpy(np.ascontiguousarray(x[lo:lo + n])).cuda())
            ys.append(torch.empty(n, dtype=torch.float64, device="cuda"))
        stream = torch.cuda.current_stream()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = sp.spmv_mcts_run_seq(plans, xs, ys, stream, fine=True, iterations=iterations, seed=7)
        wall = time.perf_counter() - t0
        k = int(np.argmin(res["time"]))
        ops, sts = res["ops"][k], res["streams"][k]
        for p in plans:
            sp.spmv_plan_set_fine(p, ops, sts)
        t_fine = sp.spmv_plan_time(plans, xs, ys, stream, 0.01, 5)
        c_ops, c_map = sp.spmv_plan_space_get(P, 2, coarse_best)
        for p in plans:
            sp.spmv_plan_reorder(p, c_ops, c_map, 2)
        t_coarse = sp.spmv_plan_time(plans, xs, ys, stream, 0.01, 5)
        count = sp.spmv_fine_count(plans[0], 2)
    finally:
        for p in plans:
            sp.spmv_plan_destroy(p)
    return {"n_tokens": int(ops.size), "programs": count, "iterations": int(res["time"].size),
            "wall_s": round(wall, 2),
            "search_best_us": round(float(res["time"].min()) * 1e6, 2),
            "search_median_us": round(float(np.median(res["time"])) * 1e6, 2),
            "best_fine_us": round(float(np.median(t_fine)) * 1e6, 2),
            "best_coarse_us": round(float(np.median(t_coarse)) * 1e6, 2),
            "best_fine_order": [sp.spmv_op_name(int(t)) + (f"@{int(s)}" if s >= 0 else "")
                                for t, s in zip(ops, sts)]}


def ranks_section(sp, torch, A, P, x, ops, smap, tune, steps: int = 100) -> dict:
    """Every rank's share of the same matrix, one after another on this GPU,
    with the chosen plan: step time and y_L per rank, and the max over ranks
    that the paper's protocol reports (Sec. III-C3)."""
    out = []
    for q in range(P):
        first = sp.spmv_plan_create(A, P, q, ops, smap, 2, tune)
        info = sp.spmv_plan_info(first)
        R = max(1, math.ceil(2 * MALL_BYTES / max(info["device_bytes"] + 16 * info["n_loc"], 1)))
        plans = [first] + [sp.spmv_plan_create(A, P, q, ops, smap, 2, tune) for _ in range(R - 1)]
        try:
            lo, n = info["lo"], info["n_loc"]
            halo = sp.spmv_plan_get_i32(first, sp.SPMV_I32_HALO_COLS).astype(np.int64)
            xs, ys = [], []
            for p in plans:
                sp.spmv_plan_inbox(p)[:] = x[halo]
                xs.append(torch.from_numpy(np.ascontiguousarray(x[lo:lo + n])).cuda())
                ys.append(torch.empty(n, dtype=torch.float64, device="cuda"))
            stream = torch.cuda.current_stream()
            for i in range(2 * R):
                sp.spmv_exec(plans[i % R], xs[i % R], ys[i % R], stream)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for i in range(steps):
                sp.spmv_exec(plans[i % R], xs[i % R], ys[i % R], stream)
            torch.cuda.synchronize()
            step_us = (time.perf_counter() - t0) / steps * 1e6
            yl_us = time_op(sp, torch, plans, sp.SPMV_OP_YL, xs, ys, max(10 * R, 200))
            B = step_bytes(info)
            out.append({"rank": q, "n_loc": n, "n_halo": info["n_halo"],
                        "form_local": info["form_local"], "step_us": round(step_us, 2),
                        "yL_us": round(yl_us, 3),
                        "yL_frac": round(B["yL"] / (yl_us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)})
        finally:
            for p in plans:
                sp.spmv_plan_destroy(p)
    return {"ranks": out, "max_step_us": max(d["step_us"] for d in out),
            "max_rank": max(out, key=lambda d: d["step_us"])["rank"]}


def stability_section(sp, A, P, r, x, replicas, ktune, first_res, repeats: int,
                      t_measure: float) -> dict:
    """How much of the design-rule output survives timing noise (Sec. IV):
    the sweep is repeated `repeats` more times on the same share, and each
    sweep's classes and rules are compared with the first one's."""
    from paper_2203_02530_amd import rules
    from paper_2203_02530_amd import tune as tuner

    def rule_out(res):
        t = np.empty(len(res))
        for d in res:
            t[d["index"]] = d["t"]
        dr = rules.design_rules(rules.plan_space(P, 2), t)
        y = np.asarray(dr["labels"]["labels"])
        fast = [rs for rs in dr["rules"] if rs["class"] == 0]
        top = max(fast, key=lambda rs: rs["samples"])["text"] if fast else []
        return t, y, top
    runs = [rule_out(first_res)]
    for _ in range(repeats):
        res = tuner.sweep_plans(A, P, r, x, 2, ktune, t_measure=t_measure, n_measure=1,
                                replicas=replicas)
        runs.append(rule_out(res))
    t0, y0, top0 = runs[0]
    fast0 = set(np.flatnonzero(y0 == 0).tolist())
    out = {"sweeps": len(runs), "n_classes": [int(np.unique(y).size) for _, y, _ in runs],
           "fastest_class_size": [int((y == 0).sum()) for _, y, _ in runs],
           "top_rules_fastest_class": [list(top) for _, _, top in runs], "vs_first": []}
    for t, y, top in runs[1:]:
        fast = set(np.flatnonzero(y == 0).tolist())
        same_k = np.unique(y).size == np.unique(y0).size
        out["vs_first"].append({
            "time_rank_corr": round(float(np.corrcoef(np.argsort(np.argsort(t0)),
                                                      np.argsort(np.argsort(t)))[0, 1]), 4),
            "same_class_count": bool(same_k),
            "label_agreement": round(float((y == y0).mean()), 4) if same_k else None,
            "fastest_class_jaccard": round(len(fast & fast0) / max(len(fast | fast0), 1), 4),
            "top_rule_set_equal": list(top) == list(top0),
            "top_rules_shared": len(set(top) & set(top0)),
            "median_time_change": round(float(np.median(np.abs(t - t0) / t0)), 4)})
    return out


def measure_share(sp, torch, gen, key: str, args, sweep: bool = True,
                  autotune: bool = False) -> tuple[dict, dict]:
    """One rank share: the plan (chosen by the cold sweep of every plan, or
    the default), timed steps, per-op event times and the host timeline of
    the chosen plan, each GPU op's duration over back-to-back launches, the
    device phase, and the roofline of the op with the most algorithmic
    bytes.  Returns (result, context for further sections)."""
    from paper_2203_02530_amd import tune as tuner
    w = gen.WORKLOADS[key]
    t0 = time.perf_counter()
    A = w["build"]()
    P, r = w["nranks"], w["rank"]
    x = w["x"](A.n_cols)
    build_s = time.perf_counter() - t0
    ktune = {"lanes_local": args.lanes, "rows_local": args.rows, "kernel_local": args.kernel,
             "chunk_local": args.chunk, "form": args.form, "width": args.width}
    ctx = {"A": A, "P": P, "r": r, "x": x, "ktune": ktune, "res": None, "best": None}
    tuned = None
    if autotune:
        # the y_L kernel variant chosen by the autotuner (stream forms, window,
        # width, summing lanes, vector lanes and rows per group), timed over
        # cold replicas; the sweep and every measurement below use it
        progress(f"{key}: kernel autotuner")
        t0 = time.perf_counter()
        kbest, kres = tuner.tune_kernel(A, P, r, x, launches=200)
        tuned = {"wall_s": round(time.perf_counter() - t0, 1), "best": kbest,
                 "results": sorted(({"tune": d["tune"], "us": round(d["us"], 3)} for d in kres),
                                   key=lambda d: d["us"])}
        ktune = {**ktune, **kbest}
        ctx["ktune"] = ktune
    ops = smap = None
    sweep_out = None
    if sweep and P > 1 and args.plan == "auto":
        R0 = args.replicas or replicas_for(A, P, r, ktune, sp)
        progress(f"{key}: plan sweep over {R0} cold replicas")
        res = tuner.sweep_plans(A, P, r, x, 2, ktune, t_measure=args.sweep_measure, n_measure=1,
                                replicas=R0)
        top = [d["index"] for d in tuner.best_plans(res, 8)]
        again = tuner.sweep_plans(A, P, r, x, 2, ktune, t_measure=args.sweep_measure,
                                  n_measure=5, indices=top, replicas=R0)
        best = tuner.best_plans(again, 1)[0]["index"]
        sweep_out = tuner.sweep_summary(res)
        sweep_out["chosen_index"] = best
        ops, smap = sp.spmv_plan_space_get(P, 2, best)
        ctx.update(res=res, best=best, R0=R0)
    elif args.plan not in ("auto", "default") and P > 1:
        ops, smap = sp.spmv_plan_space_get(P, 2, int(args.plan))
    tune = {"flags": 0, "lanes_local": args.lanes, "lanes_remote": args.lanes_remote,
            "rows_local": args.rows, "rows_remote": args.rows_remote,
            "kernel_local": args.kernel, "chunk_local": args.chunk,
            "chunk_remote": args.chunk_remote, "xcd_remap": args.xcd_remap,
            "fuse_unpack": args.fuse_unpack, "form": args.form, "width": args.width}
    if tuned:
        tune.update(tuned["best"])
    ctx["ops"], ctx["smap"], ctx["tune"] = ops, smap, tune

    progress(f"{key}: timed steps")
    first = sp.spmv_plan_create(A, P, r, ops, smap, 2, tune)
    info = sp.spmv_plan_info(first)
    lo, n = info["lo"], info["n_loc"]
    R = args.replicas or max(1, math.ceil(2 * MALL_BYTES / max(info["device_bytes"] + 16 * n, 1)))
    plans = [first] + [sp.spmv_plan_create(A, P, r, ops, smap, 2, tune) for _ in range(R - 1)]
    try:
        halo = sp.spmv_plan_get_i32(first, sp.SPMV_I32_HALO_COLS).astype(np.int64)
        xs, ys = [], []
        for p in plans:
            sp.spmv_plan_inbox(p)[:] = x[halo]
            xs.append(torch.from_numpy(np.ascontiguousarray(x[lo:lo + n])).cuda())
            ys.append(torch.empty(n, dtype=torch.float64, device="cuda"))
        stream = torch.cuda.current_stream()
        torch.cuda.synchronize()
        if args.kernel_only:
            return kernel_only(sp, torch, key, info, plans, xs, ys, stream, args), ctx

        # The timed step: the share's whole device work with its inputs (A,
        # x and the halo) resident in HBM -- Pack, y_L, Unpack, y_R on one
        # stream (spmv_exec_resident) -- rotating over the cold replicas.
        # One full exec per replica first puts each replica's halo in its
        # device receive buffer through the staged exchange.  The loop
        # passes raw addresses straight to the C entry point.
        for i in range(R):
            sp.spmv_exec(plans[i], xs[i], ys[i], stream)
        res_fn = sp._lib.spmv_exec_resident
        exec_fn = sp._lib.spmv_exec
        call = [(p, x_.data_ptr(), y_.data_ptr()) for p, x_, y_ in zip(plans, xs, ys)]
        sh = stream.cuda_stream
        for i in range(args.warmup):
            sp.spmv_exec_resident(plans[i % R], xs[i % R], ys[i % R], stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(args.steps):
            p, xp, yp = call[i % R]
            if res_fn(p, xp, yp, sh):
                raise sp.SpmvError(-5, sp.spmv_last_error())
        torch.cuda.synchronize()
        ms_step = (time.perf_counter() - t0) / args.steps * 1e3

        # The whole program with the emulated exchange (spmv_exec: the halo
        # staged through pinned host memory both ways, the plan's order and
        # streams, host-synchronous): the PCIe-inclusive rate
        for i in range(args.warmup):
            sp.spmv_exec(plans[i % R], xs[i % R], ys[i % R], stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(args.steps):
            p, xp, yp = call[i % R]
            if exec_fn(p, xp, yp, sh):
                raise sp.SpmvError(-5, sp.spmv_last_error())
        torch.cuda.synchronize()
        ms_exec = (time.perf_counter() - t0) / args.steps * 1e3

        # per-step event times inside the plan, from a separate profiled pass
        # (the event records add host work, so they stay out of the timed loop)
        for p in plans:
            sp.spmv_plan_set_profile(p, True)
            sp.spmv_plan_reset_times(p)
        for i in range(min(args.steps, 100)):
            sp.spmv_exec(plans[i % R], xs[i % R], ys[i % R], stream)
        torch.cuda.synchronize()
        ms = np.zeros(sp.SPMV_N_VERTICES + 1)
        cnt = np.zeros(sp.SPMV_N_VERTICES + 1)
        for p in plans:
            ms += sp.spmv_plan_get_f64(p, sp.SPMV_F64_OP_MS)
            cnt += sp.spmv_plan_get_f64(p, sp.SPMV_F64_OP_COUNT)
        in_plan = np.where(cnt > 0, ms / np.maximum(cnt, 1), 0.0) * 1e3
        # host timeline of the same plan (where the host waits), its own pass
        for p in plans:
            sp.spmv_plan_set_profile(p, False, host=True)
            sp.spmv_plan_reset_times(p)
        for i in range(min(args.steps, 200)):
            sp.spmv_exec(plans[i % R], xs[i % R], ys[i % R], stream)
        torch.cuda.synchronize()
        h_us = sum(sp.spmv_plan_get_f64(p, sp.SPMV_F64_HOST_US) for p in plans)
        h_n = sum(float(sp.spmv_plan_get_f64(p, sp.SPMV_F64_HOST_COUNT)[0]) for p in plans)
        for p in plans:
            sp.spmv_plan_set_profile(p, False)
        B = step_bytes(info)
        LB = launch_bytes(info)

        # each GPU op alone, back to back on one stream, events on that stream
        progress(f"{key}: kernel timings")
        launches = max(10 * R, 200)
        kern_us = {name: (time_op(sp, torch, plans, op_code(sp, name), xs, ys, launches)
                          if LB[name] > 0 else 0.0) for name in OPS}
        # the same launches of the dominant op on one replica: its arrays
        # stay in the 256 MB MALL (warm)
        op_dom = max(("yL", "yR", "pack"), key=lambda k: LB[k])
        dev_bytes = sum(LB[k] for k in OPS)     # one resident step
        grouped = info["resident_grouped"] == 1
        if grouped:
            # the step's dominant kernel is its first grouped launch (Pack,
            # y_L and y_R's slab tiles as the items of one kernel)
            kern_us["grouped"] = time_part(sp, torch, plans, 0, xs, ys, launches)
            kern_us["slab_sums"] = time_part(sp, torch, plans, 1, xs, ys, launches)
            dom, dom_variant = "grouped", grouped_variant(info)
            warm_us = time_part(sp, torch, plans[:1], 0, xs[:1], ys[:1], launches)
        else:
            dom = op_dom
            dom_variant = kernel_variant(info, dom) if dom in ("yL", "yR") else "k_gather"
            warm_us = time_op(sp, torch, plans[:1], op_code(sp, dom), xs[:1], ys[:1], launches)
        achieved = LB[dom] / (kern_us[dom] * 1e-6) / 1e9
        tr = MEASURED_TRAFFIC.get((key, dom_variant))
        traffic, traffic_src = (tr if tr else (None, None))
        ceiling = probe_ceiling(sp, torch, traffic or LB[dom])
        op_variant = kernel_variant(info, op_dom) if op_dom in ("yL", "yR") else "k_gather"
        tr = MEASURED_TRAFFIC.get((key, op_variant))
        op_roof = {"op": op_dom, "kernel": op_variant, "bytes_per_launch": LB[op_dom],
                   "avg_us": round(kern_us[op_dom], 3),
                   "achieved": round(LB[op_dom] / (kern_us[op_dom] * 1e-6) / 1e9, 2),
                   "frac": round(LB[op_dom] / (kern_us[op_dom] * 1e-6) / 1e9 / HBM_PEAK_GBS, 4),
                   "traffic": tr[0] if tr else None, "traffic_source": tr[1] if tr else None}
        gathers = None
        if op_dom == "yR" and info["form_remote"] == 5:
            # y_R in column slabs: its x gathers against the gather probe
            gathers = gather_ceiling(sp, torch, info["nnz_remote"],
                                     -(-info["n_halo"] // 8))
            gathers["yR_over_per_xcd_gathers"] = round(kern_us["yR"] / gathers["per_xcd_us"], 3)
        plan_order = [sp.spmv_op_name(int(t))
                      for t in sp.spmv_plan_get_i32(first, sp.SPMV_I32_OP_ORDER)]
        plan_streams = {sp.spmv_op_name(v): int(m) for v, m in enumerate(
            sp.spmv_plan_get_i32(first, sp.SPMV_I32_STREAM_MAP)) if m >= 0}
    finally:
        for p in plans:
            sp.spmv_plan_destroy(p)
    out = {
        "workload": w["desc"], "input_build_s": round(build_s, 1),
        "value": round(dev_bytes / (ms_step * 1e-3) / 1e9, 3), "ms_per_step": round(ms_step, 5),
        "frac_of_peak": round(dev_bytes / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "gflops": round(2.0 * (info["nnz_local"] + info["nnz_remote"]) / (ms_step * 1e-3) / 1e9, 3),
        "exec_with_staged_exchange": {
            "note": "spmv_exec: the plan's order and streams with the halo staged through "
                    "pinned host memory both ways (PCIe-inclusive; not the headline value)",
            "ms_per_step": round(ms_exec, 5),
            "gbs": round(B["total"] / (ms_exec * 1e-3) / 1e9, 3),
            "host_link_bytes": B["host_link"]},
        "config": {"workload": w["desc"], "rows": int(A.n_rows), "nnz": int(A.nnz),
                   "nranks": P, "rank": r, "n_loc": n, "nnz_local": info["nnz_local"],
                   "nnz_remote": info["nnz_remote"], "n_halo": info["n_halo"],
                   "n_send": info["n_send"], "n_remote_rows": info["n_remote_rows"],
                   "plan": args.plan if sweep_out is None else "auto",
                   "kernel_yL": kernel_variant(info, "yL"), "kernel_yR": kernel_variant(info, "yR"),
                   "form_local": info["form_local"], "form_remote": info["form_remote"],
                   "n_tiles_local": info["n_tiles_local"], "n_tiles_remote": info["n_tiles_remote"],
                   "xcd_remap": info["xcd_remap"], "fuse_unpack": info["fuse_unpack"],
                   "fused_combine": info["fused_combine"], "replicas": R,
                   "step": {1: "y_R's column-slab tiles, then y_L and Pack, as one grouped "
                                   "launch, then the slab sums into y",
                            3: "one launch: y_L, Pack as extra blocks, each remote row's "
                               "sum added where its local sum is stored",
                            2: "y_L with Pack as extra blocks of its launch, then y_R into y",
                            0: "Pack, y_L, Unpack, y_R, one launch each"}.get(
                                info["resident_grouped"], "see spmv_exec_resident") +
                           ", on one stream, halo resident in HBM (spmv_exec_resident)",
                   "resident_grouped": info["resident_grouped"],
                   "step_device_bytes": dev_bytes, "exec_device_bytes": B["total"],
                   "exec_host_link_bytes": B["host_link"]},
        "roofline": {"bound": "hbm", "kernel": f"{dom} {dom_variant}",
                     "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "traffic_source": traffic_src,
                     "traffic_over_algorithmic": round(traffic / LB[dom], 3) if traffic else None,
                     "traffic_gbs": (round(traffic / (kern_us[dom] * 1e-6) / 1e9, 1)
                                     if traffic else None),
                     "bytes_per_launch": LB[dom], "avg_us": round(kern_us[dom], 3),
                     "launches": launches,
                     **({"items": "Pack, y_L and y_R's column-slab tiles"} if grouped else {})},
        "op_roofline": op_roof,
        "warm": {"kernel": dom, "avg_us": round(warm_us, 3),
                 "achieved": round(LB[dom] / (warm_us * 1e-6) / 1e9, 1),
                 "note": "one replica, launched back to back: its arrays stay in the MALL"},
        "gather_probe": gathers,
        "hbm_probe": {**ceiling, "kernel_moved_over_probe": (
            round(traffic / (kern_us[dom] * 1e-6) / 1e9 / ceiling["read_gbs"], 3)
            if traffic else None)},
        "step_bytes": dev_bytes,
        "kernel_us": {k: round(float(v), 3) for k, v in kern_us.items()},
        "kernel_bytes": LB,
        "kernel_gbs": {k: round(LB[k] / (kern_us[k] * 1e-6) / 1e9, 1) for k in kern_us
                       if kern_us[k] > 0 and LB[k] > 0},
        "in_plan_event_us": {"pack": round(float(in_plan[sp.SPMV_OP_PACK]), 3),
                             "yL": round(float(in_plan[sp.SPMV_OP_YL]), 3),
                             "unpack": round(float(in_plan[sp.SPMV_OP_UNPACK]), 3),
                             "yR": round(float(in_plan[sp.SPMV_OP_YR]), 3),
                             "combine": round(float(in_plan[sp.SPMV_N_VERTICES]), 3),
                             "post_send_copy": round(float(in_plan[sp.SPMV_OP_POST_SEND]), 3),
                             "post_recv_copy": round(float(in_plan[sp.SPMV_OP_POST_RECV]), 3)},
        "host_timeline_us": [[name, round(float(t) / max(h_n, 1.0), 2)]
                             for name, t in zip(plan_order, h_us)],
        "plan_sweep": sweep_out, "plan_order": plan_order, "plan_streams": plan_streams,
        "kernel_autotune": tuned,
    }
    ctx["info"] = info
    return out, ctx


def kernel_only(sp, torch, key, info, plans, xs, ys, stream, args) -> dict:
    """Counter runs: one op launched back to back over the cold replicas,
    then a plain copy of known size whose FETCH_SIZE / WRITE_SIZE readings
    calibrate the counters."""
    LB = launch_bytes(info)
    name = args.op or ("grouped" if info["resident_grouped"] == 1
                       else max(("yL", "yR", "pack"), key=lambda k: LB[k]))
    launches = max(10 * len(plans), 200)
    if name in ("grouped", "slab_sums"):
        # a resident step's halo: one full exec per replica first
        for i in range(len(plans)):
            sp.spmv_exec(plans[i], xs[i], ys[i], stream)
        us = time_part(sp, torch, plans, 0 if name == "grouped" else 1, xs, ys, launches)
    else:
        us = time_op(sp, torch, plans, op_code(sp, name), xs, ys, launches)
    gathers = None
    if name == "yR" and info["form_remote"] == 5:
        # the gather probe beside y_R in column slabs (per XCD, then over
        # the whole halo), for counters of the same gathers without rows
        gathers = gather_ceiling(sp, torch, info["nnz_remote"], -(-info["n_halo"] // 8),
                                 launches=20)
    nbytes = 64 << 20
    src = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").normal_()
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(10):
        sp.spmv_hbm_probe(1, src, dst, nbytes, 0, stream)
    torch.cuda.synchronize()
    return {"kernel_only": True, "workload": key, "op": name,
            "variant": (kernel_variant(info, name) if name in ("yL", "yR") else
                        grouped_variant(info) if name in ("grouped", "slab_sums") else "k_gather"),
            "avg_us": round(us, 3), "launches": launches + 2 * len(plans),
            "bytes_per_launch": LB[name], "copy_bytes_each_way": nbytes, "copy_launches": 10,
            "gather_probe": gathers}


def extra_summary(out: dict) -> dict:
    """The fields of a share carried beside the headline."""
    rf = out["roofline"]
    return {"workload": out["workload"], "kernel": rf["kernel"],
            "bytes_per_launch": rf["bytes_per_launch"], "avg_us": rf["avg_us"],
            "achieved": rf["achieved"], "frac": rf["frac"], "traffic": rf["traffic"],
            "traffic_source": rf["traffic_source"], "step_us": round(out["ms_per_step"] * 1e3, 2),
            "value": out["value"], "frac_of_peak": out["frac_of_peak"],
            "exec_with_staged_exchange": out["exec_with_staged_exchange"],
            "hbm_probe": out["hbm_probe"],
            "kernel_us": out["kernel_us"], "plan_sweep": out["plan_sweep"],
            "kernel_autotune": out["kernel_autotune"], "config": out["config"]}


def paper_section(sp, torch, gen, tuner) -> dict:
    """The paper's own workload (Sec. IV: banded 150,000 x 150,000, 10
    entries per row in half-bandwidth 37,500, P = 4): every plan of rank 1's
    share timed cold, and the design-rule pipeline on those times."""
    w = gen.WORKLOADS["banded_150k_p4r1"]
    A = w["build"]()
    P, r = w["nranks"], w["rank"]
    x = w["x"](A.n_cols)
    R0 = replicas_for(A, P, r, {}, sp)
    t0 = time.perf_counter()
    res = tuner.sweep_plans(A, P, r, x, 2, {}, t_measure=0.01, n_measure=1, replicas=R0)
    wall = time.perf_counter() - t0
    out = {"workload": w["desc"], "replicas": R0, "sweep_s": round(wall, 1),
           "plan_sweep": tuner.sweep_summary(res)}
    out["design_rules"] = rules_section(sp, torch, A, P, r, x, res, R0, {}, live=False)
    return out


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default=HEADLINE)
    ap.add_argument("--replicas", type=int, default=0, help="0 = enough to exceed 2x MALL")
    ap.add_argument("--plan", default="auto",
                    help="'auto' (sweep the design space, keep the fastest), 'default', "
                         "or a plan-space index")
    ap.add_argument("--sweep-measure", type=float, default=0.01,
                    help="seconds per measurement in the plan sweep (paper: 0.01)")
    ap.add_argument("--lanes", type=int, default=0)
    ap.add_argument("--lanes-remote", type=int, default=0)
    ap.add_argument("--rows", type=int, default=0)
    ap.add_argument("--rows-remote", type=int, default=0)
    ap.add_argument("--kernel", type=int, default=0, help="0 auto, 1 vector CSR, 2 stream CSR")
    ap.add_argument("--chunk", type=int, default=0)
    ap.add_argument("--chunk-remote", type=int, default=0)
    ap.add_argument("--width", type=int, default=0, help="stream CSR entries per load (0 auto)")
    ap.add_argument("--form", type=int, default=0,
                    help="stream form: 0 auto, 1 packed tiles, 2 sliced ELL, 3 sliced ELL with "
                         "16-bit column offsets, 4 packed tiles with 16-bit columns, 5 y_R in "
                         "column slabs")
    ap.add_argument("--xcd-remap", type=int, default=0)
    ap.add_argument("--fuse-unpack", type=int, default=0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-rules", action="store_true",
                    help="skip the design-space stages on the 7-point share and the paper's "
                         "workload")
    ap.add_argument("--extras", type=int, default=1,
                    help="also measure the 7-point and 27-point stencil shares (1 = yes)")
    ap.add_argument("--stability", type=int, default=2,
                    help="repeated sweeps of the 7-point share for the rule stability figure")
    ap.add_argument("--batch-shares", type=int, default=64,
                    help="rank shares in the batched section (0 = skip it)")
    ap.add_argument("--serve-requests", type=int, default=20000,
                    help="requests in the serving section (0 = skip it)")
    ap.add_argument("--all-ranks", type=int, default=1,
                    help="run every rank's share of the 7-point matrix with the chosen plan "
                         "and report the max over ranks (1 = yes)")
    ap.add_argument("--tune-kernel", action="store_true",
                    help="also time the product kernel variants of the autotuner on the "
                         "headline share (y_L and y_R)")
    ap.add_argument("--kernel-only", action="store_true",
                    help="only launch one op of the workload back-to-back and the copy probe "
                         "of known size (for hardware-counter runs), print their timings")
    ap.add_argument("--batch-device-only", action="store_true",
                    help="only run the device phase of the batch of --batch-shares power-law "
                         "shares (no staging), --steps times (for profiler runs)")
    ap.add_argument("--batch-opts", default="{}",
                    help="batch options for --batch-device-only, as JSON")
    ap.add_argument("--op", default="", help="op for --kernel-only (pack, yL, unpack, yR, "
                                             "grouped, slab_sums; default: the grouped "
                                             "launch where the resident step is grouped, "
                                             "else the op with the most bytes)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one rank share on one GPU; --gpus {args.gpus} is not "
              "supported (the library runs one rank's share per GPU; the multi-GPU "
              "exchange is not implemented)", file=sys.stderr)
        return 2

    import torch
    import gen
    import paper_2203_02530_amd as sp

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)

    if args.kernel_only:
        out, _ = measure_share(sp, torch, gen, args.workload, args, sweep=False)
        print(json.dumps(out), flush=True)
        return 0
    if args.batch_device_only:
        print(json.dumps(batch_device_only(sp, torch, gen, args.batch_shares, args.steps,
                                           json.loads(args.batch_opts))), flush=True)
        return 0

    head, hctx = measure_share(sp, torch, gen, args.workload, args)
    cpu = plain = None
    if not args.no_cpu:
        progress("cpu baselines")
        dyn = args.workload.startswith("powerlaw")
        B = float(head["config"]["step_device_bytes"])   # the same bytes as the step
        cpu = cpu_baseline(hctx["A"], hctx["P"], hctx["r"], hctx["x"], B, dyn)
        plain = cpu_plain(hctx["A"], hctx["P"], hctx["r"], hctx["x"], B, dyn)
    kernel_tune = None
    if args.tune_kernel:
        from paper_2203_02530_amd import tune as tuner
        progress("kernel autotuner")
        t0 = time.perf_counter()
        A, P, r, x = hctx["A"], hctx["P"], hctx["r"], hctx["x"]
        bl, rl = tuner.tune_kernel(A, P, r, x, launches=200)
        br, rr = tuner.tune_kernel(A, P, r, x, candidates=tuner.DEFAULT_REMOTE_CANDIDATES,
                                   launches=200, op=sp.SPMV_OP_YR)
        kernel_tune = {"wall_s": round(time.perf_counter() - t0, 1),
                       "yL": {"best": bl, "results": [{"tune": d["tune"], "us": round(d["us"], 3)}
                                                      for d in rl]},
                       "yR": {"best": br, "results": [{"tune": d["tune"], "us": round(d["us"], 3)}
                                                      for d in rr]}}
    del hctx
    batched = serving = None
    if args.batch_shares > 0:
        progress("batched shares")
        batched = batched_section(sp, torch, gen, args.batch_shares, reps=4)
    if args.serve_requests > 0:
        progress("serving")
        serving = serving_section(sp, torch, gen, args.serve_requests, 5000.0, 128)

    extras = {}
    design = None
    if args.extras:
        for key in EXTRAS:
            ex, ctx = measure_share(sp, torch, gen, key, args,
                                    autotune=key == "stencil27_150_p8r3")
            extras[key] = extra_summary(ex)
            if key == "laplace3d_128_p4r1" and not args.no_rules and ctx["res"] is not None:
                A, P, r, x = ctx["A"], ctx["P"], ctx["r"], ctx["x"]
                progress(f"{key}: design rules")
                design = {"workload": ex["workload"],
                          "rules": rules_section(sp, torch, A, P, r, x, ctx["res"], ctx["R0"],
                                                 ctx["ktune"])}
                if args.stability > 0:
                    progress(f"{key}: rule stability ({args.stability} more sweeps)")
                    design["stability"] = stability_section(
                        sp, A, P, r, x, ctx["R0"], ctx["ktune"], ctx["res"], args.stability,
                        args.sweep_measure)
                progress(f"{key}: fine-grained search")
                design["fine_grained"] = fine_section(sp, torch, A, P, r, x, ctx["R0"],
                                                      ctx["ktune"], ctx["best"])
                if args.all_ranks:
                    progress(f"{key}: every rank's share")
                    design["all_ranks"] = ranks_section(sp, torch, A, P, x, ctx["ops"],
                                                        ctx["smap"], ctx["tune"])
            del ctx
    paper = None
    if args.plan == "auto" and not args.no_rules:
        from paper_2203_02530_amd import tune as tuner
        progress("the paper's workload")
        paper = paper_section(sp, torch, gen, tuner)

    out = {
        "metric": "rank-share SpMV GB/s vs HBM peak; batched req/s + p50/p99 latency vs plain",
        "value": head["value"],
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": head["config"],
        "roofline": head["roofline"],
        "op_roofline": head["op_roofline"],
        "cpu_baseline": cpu,
        "cpu_plain": plain,
        "frac_of_peak": head["frac_of_peak"],
        "exec_with_staged_exchange": head["exec_with_staged_exchange"],
        "warm": head["warm"],
        "hbm_probe": head["hbm_probe"],
        "gather_probe": head["gather_probe"],
        "gflops": head["gflops"],
        "kernel_us": head["kernel_us"],
        "kernel_bytes": head["kernel_bytes"],
        "kernel_gbs": head["kernel_gbs"],
        "in_plan_event_us": head["in_plan_event_us"],
        "host_timeline_us": head["host_timeline_us"],
        "plan_sweep": head["plan_sweep"],
        "plan_order": head["plan_order"],
        "plan_streams": head["plan_streams"],
        "kernel_tune": kernel_tune,
        "batched": batched,
        "serving": serving,
        "extras": extras,
        "design_space": design,
        "paper_workload": paper,
    }
    progress("done")
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
