"""Batched execution: many rank shares in grouped persistent kernels, as
stream launches or one hipGraph, with the staging pipelined over chunks of
shares.  Each share's y must be bit-identical to its own spmv_exec (same
tiles, same device code), and within tolerance of the oracle; halo buffers
bit-exact; every replay equal to the eager result."""
import numpy as np
import pytest

import gen
import oracle
import paper_2203_02530_amd as sp
from gpu_util import bits, log, run_share

pytestmark = pytest.mark.gpu
TUNE = {"kernel_local": 2, "kernel_remote": 2, "chunk_local": 8, "chunk_remote": 8, "width": 2,
        "form": 1}


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch
    assert torch.cuda.is_available()
    oracle.build(force=False)
    yield


def _shares():
    out = []
    for s in range(3):
        A = gen.power_law(20000, seed=4000 + s)
        out.append((A, 16, 5, gen.x_normal(A.n_cols, 4100 + s)))
    A = gen.banded_uniform(6000, 10, 1500, seed=11)
    out.append((A, 4, 1, gen.x_normal(A.n_cols, 12)))
    A = gen.laplacian_3d7(16)
    out.append((A, 4, 1, gen.x_uniform(A.n_cols, 2)))
    A = gen.laplacian_2d5(64)
    out.append((A, 1, 0, gen.x_uniform(A.n_cols, 1)))
    A = gen.laplacian_2d5(2, 2)
    out.append((A, 6, 5, gen.x_normal(4, 3)))          # empty share
    A = gen.stencil_3d27(12, seed=3)
    out.append((A, 8, 3, gen.x_normal(A.n_cols, 30)))
    A = gen.power_law(12000, mean_len=300.0, seed=44)  # rows longer than the window
    out.append((A, 4, 1, gen.x_normal(A.n_cols, 45)))
    return out


def _setup(shares, tune=TUNE):
    import torch
    plans, xs, ys, refs, solo = [], [], [], [], []
    for A, P, r, x in shares:
        ref = oracle.share_reference(A, P, r, x)
        res, _ = run_share(A, P, r, x, tune=tune, ref=ref, keep_plan=True)
        p = res.pop("plan")
        info = res["info"]
        lo, n = info["lo"], info["n_loc"]
        plans.append(p)
        xs.append(torch.from_numpy(x[lo:lo + n].copy()).cuda() if n else None)
        ys.append(torch.full((n,), float("nan"), dtype=torch.float64, device="cuda") if n else None)
        refs.append(ref)
        solo.append(res)
    return plans, xs, ys, refs, solo


def _check(plans, ys, refs, solo):
    for i, (p, y, ref, res) in enumerate(zip(plans, ys, refs, solo)):
        if y is None:
            continue
        yb = y.cpu().numpy()
        assert np.array_equal(bits(yb), bits(res["y"])), i
        assert oracle.within_tolerance(yb, ref["y"], ref["absax"]).all(), i
        assert np.array_equal(bits(sp.spmv_plan_outbox(p)), bits(ref["sendbuf"])), i
        assert np.array_equal(bits(sp.spmv_plan_get_f64(p, sp.SPMV_F64_X_HALO)),
                              bits(ref["inbox"])), i


@pytest.mark.parametrize("opts", [{"use_graph": 1}, {"use_graph": 2},
                                  {"use_graph": 1, "xcd_affinity": 1, "blocks_per_cu": 2},
                                  {"use_graph": 2, "xcd_affinity": 2, "blocks_per_cu": 1},
                                  {"use_graph": 2, "copy_streams": 1},
                                  {"use_graph": 2, "copy_streams": 3},
                                  {"use_graph": 2, "chunks": 1},
                                  {"use_graph": 2, "chunks": 3},
                                  {"use_graph": 1, "chunks": 4},
                                  {"use_graph": 2, "chunks": 9, "copy_streams": 2},
                                  {"use_graph": 1, "chunks": 200},
                                  {"use_graph": 2, "persistent": 1},
                                  {"use_graph": 1, "persistent": 1, "chunks": 3},
                                  {"use_graph": 2, "persistent": 2, "xcd_affinity": 1}])
def test_batch_bit_identical_to_solo(opts):
    import torch
    log(f"batch opts {opts}")
    shares = _shares()
    plans, xs, ys, refs, solo = _setup(shares)
    try:
        b = sp.spmv_batch_create(plans, opts)
        try:
            info = sp.spmv_batch_info(b)
            assert info["n_shares"] == len(plans) and sum(info["n_items"]) > 0
            want = min(opts.get("chunks", 0), len(plans)) or max(1, len(plans) // 8)
            assert info["n_chunks"] == want, info
            assert info["persistent"] == (1 if opts.get("persistent") == 1 else 0)
            for rep in range(3):
                for y in ys:
                    if y is not None:
                        y.fill_(float("nan"))          # eager work between replays
                torch.cuda.synchronize()
                sp.spmv_batch_exec(b, xs, ys, torch.cuda.current_stream())
                _check(plans, ys, refs, solo)
        finally:
            sp.spmv_batch_destroy(b)
    finally:
        for p in plans:
            sp.spmv_plan_destroy(p)


@pytest.mark.parametrize("use_graph", [1, 2])
def test_batch_with_16bit_tiles(use_graph):
    """Shares whose local product uses packed tiles with 16-bit columns (and
    shares whose columns do not fit, in 32-bit tiles) in one batch."""
    import torch
    shares = _shares()
    plans, xs, ys, refs, solo = _setup(shares, tune={**TUNE, "form": 4})
    try:
        forms = [sp.spmv_plan_info(p)["form_local"] for p in plans]
        assert 4 in forms
        b = sp.spmv_batch_create(plans, {"use_graph": use_graph})
        try:
            for rep in range(2):
                for y in ys:
                    if y is not None:
                        y.fill_(float("nan"))
                torch.cuda.synchronize()
                sp.spmv_batch_exec(b, xs, ys, torch.cuda.current_stream())
                _check(plans, ys, refs, solo)
        finally:
            sp.spmv_batch_destroy(b)
    finally:
        for p in plans:
            sp.spmv_plan_destroy(p)


@pytest.mark.parametrize("opts", [{"use_graph": 2}, {"use_graph": 1, "chunks": 3},
                                  {"use_graph": 2, "chunks": 9, "xcd_affinity": 2},
                                  {"use_graph": 2, "chunks": 2, "persistent": 1,
                                   "blocks_per_cu": 1},
                                  {"use_graph": 1, "persistent": 1, "xcd_affinity": 1}])
def test_batch_with_column_slabs(opts):
    """Shares whose y_R runs in column slabs (slab tiles on their slab's XCD,
    then the slab sums) batched with shares in packed tiles: every share
    bit-identical to its own exec, over repeated runs."""
    import torch
    log(f"batch with column slabs {opts}")
    shares = _shares()
    # form 5 leaves y_L automatic: the 7-point share would go sliced (not
    # batchable), so it keeps packed tiles here
    slab = {0, 2, 3, 7, 8}
    plans, xs, ys, refs, solo = [], [], [], [], []
    try:
        for i, sh in enumerate(shares):
            p_, x_, y_, r_, s_ = _setup([sh], tune={**TUNE, "form": 5} if i in slab else TUNE)
            plans += p_
            xs += x_
            ys += y_
            refs += r_
            solo += s_
        forms = [sp.spmv_plan_info(p)["form_remote"] for p in plans]
        assert forms.count(5) >= 4 and 1 in forms, forms
        b = sp.spmv_batch_create(plans, opts)
        try:
            for rep in range(3):
                for y in ys:
                    if y is not None:
                        y.fill_(float("nan"))
                torch.cuda.synchronize()
                sp.spmv_batch_exec(b, xs, ys, torch.cuda.current_stream())
                _check(plans, ys, refs, solo)
        finally:
            sp.spmv_batch_destroy(b)
    finally:
        for p in plans:
            sp.spmv_plan_destroy(p)


def test_batch_autotuner():
    """The batch autotuner times every candidate; every candidate gives the
    solo bits, and the options it returns are the fastest."""
    from paper_2203_02530_amd import tune as tuner
    shares = _shares()
    plans, xs, ys, refs, solo = _setup(shares)
    try:
        cands = [{"use_graph": 2, "copy_streams": 1, "blocks_per_cu": 4},
                 {"use_graph": 2, "copy_streams": 2, "blocks_per_cu": 8},
                 {"use_graph": 1, "blocks_per_cu": 8}]
        best, res = tuner.tune_batch(plans, xs, ys, candidates=cands, reps=2)
        assert [d["opts"] for d in res] == cands and all(d["ms"] > 0 for d in res)
        assert best == min(res, key=lambda d: d["ms"])["opts"]
        _check(plans, ys, refs, solo)
    finally:
        for p in plans:
            sp.spmv_plan_destroy(p)


def test_batch_same_alone_and_in_mix():
    """A share's bits do not depend on which other shares are batched with it."""
    import torch
    shares = _shares()
    plans, xs, ys, refs, solo = _setup(shares)
    try:
        out = {}
        for subset in ([0], [0, 1, 2], list(range(len(plans)))):
            b = sp.spmv_batch_create([plans[i] for i in subset])
            try:
                sp.spmv_batch_exec(b, [xs[i] for i in subset], [ys[i] for i in subset],
                                   torch.cuda.current_stream())
                out[len(subset)] = bits(ys[0].cpu().numpy())
            finally:
                sp.spmv_batch_destroy(b)
        assert np.array_equal(out[1], out[3]) and np.array_equal(out[1], out[len(plans)])
    finally:
        for p in plans:
            sp.spmv_plan_destroy(p)


def test_batch_rejects_mixed_configs():
    A = gen.laplacian_3d7(12)
    p1 = sp.spmv_plan_create(A, 2, 0, tune=TUNE)
    p2 = sp.spmv_plan_create(A, 2, 1, tune={**TUNE, "chunk_local": 4})
    p3 = sp.spmv_plan_create(A, 2, 1, tune={"kernel_local": 1})
    p4 = sp.spmv_plan_create(A, 2, 1, tune={**TUNE, "form": 2})     # sliced: no tiles
    assert sp.spmv_plan_info(p4)["form_local"] == 2
    p5 = sp.spmv_plan_create(A, 2, 1, tune={**TUNE, "form": 3})
    assert sp.spmv_plan_info(p5)["form_local"] == 3
    p6 = sp.spmv_plan_create(A, 2, 1, tune={**TUNE, "form": 4})
    assert sp.spmv_plan_info(p6)["form_local"] == 4
    try:
        sp.spmv_batch_destroy(sp.spmv_batch_create([p1, p6]))   # 16-bit tiles may join
        for bad in ([p1, p2], [p1, p3], [p1, p4], [p1, p5]):
            with pytest.raises(sp.SpmvError) as e:
                sp.spmv_batch_create(bad)
            assert e.value.code == sp.SPMV_EINVAL
        for opts in ({"copy_streams": 5}, {"copy_streams": -1}, {"use_graph": 3},
                     {"chunks": -1}, {"chunks": 257}, {"persistent": 3}):
            with pytest.raises(sp.SpmvError) as e:
                sp.spmv_batch_create([p1], opts)
            assert e.value.code == sp.SPMV_EINVAL
    finally:
        for p in (p1, p2, p3, p4, p5, p6):
            sp.spmv_plan_destroy(p)
    # y_R in column slabs of 256 / lanes rows joins a batch, as does y_R in
    # packed tiles (and y_L in 16-bit tiles either way); wide slab tiles
    # (rows per thread > 1) do not
    B = gen.power_law(20000, seed=3)
    q4 = sp.spmv_plan_create(B, 4, 1, tune={**TUNE, "form": 4})
    q5 = sp.spmv_plan_create(B, 4, 1, tune={**TUNE, "form": 5})
    qw = sp.spmv_plan_create(B, 4, 1, tune={**TUNE, "form": 5, "rows_remote": 4})
    try:
        i4, i5 = sp.spmv_plan_info(q4), sp.spmv_plan_info(q5)
        assert (i4["form_local"], i4["form_remote"]) == (4, 1)
        assert (i5["form_local"], i5["form_remote"]) == (4, 5)
        sp.spmv_batch_destroy(sp.spmv_batch_create([q4, q5]))
        with pytest.raises(sp.SpmvError) as e:
            sp.spmv_batch_create([q4, qw])
        assert e.value.code == sp.SPMV_EINVAL
    finally:
        for q in (q4, q5, qw):
            sp.spmv_plan_destroy(q)
