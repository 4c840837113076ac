"""GPU parity of the rank-share SpMV against the CPU oracle, through the C ABI.

Bar: send buffer, receive buffer and halo bit-exact; y within
1e-12 * (|A||x|)_i per row; integer-valued stencil products bit-exact; every
plan of the design space bit-identical to every other.
"""
import numpy as np
import pytest

import gen
import oracle
import paper_2203_02530_amd as sp
from gpu_util import assert_share_parity, bits, log, run_share

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    oracle.build(force=False)
    yield


# ------------------------------------------------------------ single rank

def test_laplace2d_64_single_rank():
    A = gen.laplacian_2d5(64)
    x = gen.x_uniform(A.n_cols, 1)
    log("laplace2d 64x64 P=1 uniform x")
    res, ref = run_share(A, 1, 0, x)
    assert res["info"]["n_halo"] == 0 and res["info"]["n_ops"] == 3
    assert_share_parity(res, ref)


@pytest.mark.parametrize("xkind", ["ones", "integer"])
def test_laplace_integer_vectors_bit_exact(xkind):
    for A, P, r in [(gen.laplacian_2d5(64), 1, 0), (gen.laplacian_3d7(32), 4, 1)]:
        x = np.ones(A.n_cols) if xkind == "ones" else gen.x_integer(A.n_cols, 7)
        log(f"integer vector {xkind} n={A.n_rows} P={P}")
        res, ref = run_share(A, P, r, x)
        assert np.array_equal(bits(res["y"]), bits(ref["y"]))


# ------------------------------------------------------------ multi rank

CASES = [
    ("laplace3d_16_p4", lambda: gen.laplacian_3d7(16), 4, [0, 1, 3], lambda n: gen.x_uniform(n, 2)),
    ("banded_3000_p4", lambda: gen.banded_uniform(3000, 10, 750, seed=100), 4, [0, 1, 2, 3],
     lambda n: gen.x_normal(n, 101)),
    ("stencil27_12_p8", lambda: gen.stencil_3d27(12, seed=3), 8, [0, 3, 7],
     lambda n: gen.x_normal(n, 30)),
    ("powerlaw_20k_p16", lambda: gen.power_law(20000, seed=4000), 16, [0, 5, 15],
     lambda n: gen.x_normal(n, 4100)),
    ("ragged_1001_p3", lambda: gen.banded_random(1001, seed=9), 3, [0, 1, 2],
     lambda n: gen.x_normal(n, 11)),
]


@pytest.mark.parametrize("name,build,P,ranks,xf", CASES, ids=[c[0] for c in CASES])
def test_share_default_plan(name, build, P, ranks, xf):
    A = build()
    x = xf(A.n_cols)
    for r in ranks:
        log(f"{name} rank {r}")
        res, ref = run_share(A, P, r, x)
        assert_share_parity(res, ref)


@pytest.mark.parametrize("lanes", [1, 2, 4, 8, 16, 32, 64])
@pytest.mark.parametrize("rows", [1, 2, 4, 8])
def test_lane_variants(lanes, rows):
    A = gen.power_law(30000, seed=17)
    x = gen.x_normal(A.n_cols, 18)
    log(f"power-law 30k lanes={lanes} rows={rows}")
    for fuse, remap, flags in ((2, 1, 0), (1, 2, sp.SPMV_F_NO_BUFFER)):
        res, ref = run_share(A, 4, 2, x, tune={"kernel_local": 1, "kernel_remote": 1,
                                               "lanes_local": lanes, "lanes_remote": lanes,
                                               "rows_local": rows, "rows_remote": rows,
                                               "xcd_remap": remap, "fuse_unpack": fuse,
                                               "flags": flags})
        assert_share_parity(res, ref)


@pytest.mark.parametrize("chunk", [4, 8, 16])
@pytest.mark.parametrize("width", [2, 4])
@pytest.mark.parametrize("lanes", [1, 2, 4, 8, 16])
def test_stream_variants(chunk, width, lanes):
    """Stream CSR on uneven rows, including rows longer than the window."""
    log(f"stream chunk={chunk} width={width} lanes={lanes}")
    for A, P, r, seed in [(gen.power_law(30000, seed=17), 4, 2, 18),
                          (gen.power_law(12000, mean_len=300.0, seed=44), 4, 1, 45)]:
        x = gen.x_normal(A.n_cols, seed)
        for fuse, remap in ((2, 1), (1, 2)):
            res, ref = run_share(A, P, r, x, tune={
                "kernel_local": 2, "kernel_remote": 2, "chunk_local": chunk,
                "chunk_remote": chunk, "width": width, "lanes_local": lanes,
                "lanes_remote": lanes, "xcd_remap": remap, "fuse_unpack": fuse})
            assert res["info"]["kernel_local"] == 2
            assert_share_parity(res, ref)


@pytest.mark.parametrize("chunk", [0, 4, 8, 16])
def test_sliced_form(chunk):
    """Sliced ELL against the oracle: stencils (integer x bit-exact), banded
    rows, slices cut by the end of the rows, the remote product over
    compressed rows, y_R fused or combined, and the fall back to packed
    tiles when padding would exceed 15% (uneven rows)."""
    log(f"sliced form chunk={chunk}")
    cases = [(gen.laplacian_3d7(48), 4, 1, 3),
             (gen.stencil_3d27(30, seed=5), 4, 2, 6),
             (gen.banded_uniform(60000, 10, 15000, seed=8), 4, 3, 9),
             (gen.laplacian_2d5(40), 2, 1, 10),
             (gen.laplacian_2d5(37, 29), 1, 0, 12),                # 1073 rows: ragged last slice
             (gen.banded_random(50000, 5, 27, 2000, seed=13), 1, 0, 11),   # uneven: packed tiles
             (gen.power_law(30000, seed=17), 4, 2, 18)]
    for A, P, r, seed in cases:
        x = gen.x_normal(A.n_cols, seed)
        ref = oracle.share_reference(A, P, r, x)
        split = oracle.split(A, P, r)
        for plan in (0, 5):
            ops, smap = sp.spmv_plan_space_get(P, 2, plan) if P > 1 else (None, None)
            res, _ = run_share(A, P, r, x, ops, smap, tune={
                "kernel_local": 2, "kernel_remote": 2, "chunk_local": chunk,
                "chunk_remote": chunk, "form": 2}, ref=ref)
            assert_share_parity(res, ref)
        # sliced exactly when padding stays within 15% of the entries
        rp = split["L_ptr"]
        lens = np.diff(rp)
        n = lens.size
        widths = [lens[i:i + 64].max() for i in range(0, n, 64)] if n else []
        padded = 64 * int(np.sum(widths))
        expect = 2 if n and padded <= 1.15 * max(int(rp[-1]), 1) else 1
        assert res["info"]["form_local"] == expect, (A.n_rows, padded, rp[-1])
    for A, P, r in [(gen.laplacian_3d7(32), 4, 1), (gen.laplacian_2d5(64), 1, 0)]:
        x = gen.x_integer(A.n_cols, 9)
        res, ref = run_share(A, P, r, x, tune={"kernel_local": 2, "kernel_remote": 2,
                                               "chunk_local": chunk, "form": 2})
        assert res["info"]["form_local"] == 2
        assert np.array_equal(bits(res["y"]), bits(ref["y"]))


def _expected_form(split, ask):
    """The stream form a y_L product takes (host rule): 2 when padding each
    slice of 64 rows to its widest row stays within 15% of the entries; 3
    (when asked for, or automatic) when one width for every slice fits that
    too and every column lies within 32767 of its row; packed tiles
    otherwise, 4 (asked for, or automatic) when every column lies within
    16 bits of its tile's first row (decided here with the 256-row margin
    of a tile: the cases below stay clear of the edge)."""
    rp, col = np.asarray(split["L_ptr"]), np.asarray(split["L_col"])
    lens = np.diff(rp)
    n = lens.size
    rows = np.repeat(np.arange(n), lens)
    dmax = int(np.abs(col - rows).max()) if rows.size else 0
    tile_fits = dmax <= 32767 - 256
    assert tile_fits or dmax > 32767 + 256
    packed = 4 if ask in (0, 4) and tile_fits else 1
    if ask in (1, 4):
        return packed
    if not n:
        return 2                             # no rows: width 0 keeps 32-bit columns
    widths = np.array([lens[i:i + 64].max() for i in range(0, n, 64)])
    budget = 1.15 * max(int(rp[-1]), 1)
    if 64 * int(widths.sum()) > budget:
        return packed
    uniform = 64 * int(widths.max()) * widths.size <= budget
    fits = dmax <= 32767 and int(widths.max()) > 0
    if ask == 0:
        return (3 if fits else 2) if uniform and widths.max() <= 8 else packed
    return 3 if ask == 3 and uniform and fits else 2


@pytest.mark.parametrize("chunk,width,lanes", [(0, 0, 0), (4, 2, 1), (8, 4, 2), (16, 2, 4)])
def test_packed16_form(chunk, width, lanes):
    """Packed tiles with 16-bit columns relative to each tile's first row
    against the oracle, and bit for bit against 32-bit packed tiles (same
    tiles, same order): stencils, banded rows with offsets near the 16-bit
    limit, rows longer than a window, and the fall back to 32-bit columns."""
    log(f"packed16 form chunk={chunk} width={width} lanes={lanes}")
    cases = [(gen.stencil_3d27(30, seed=5), 4, 2, 6),
             (gen.laplacian_3d7(48), 4, 1, 3),
             (gen.banded_uniform(90000, 4, 32000, seed=2), 1, 0, 4),   # offsets up to 32,000
             (gen.banded_uniform(2000, 1500, 2000, seed=7), 1, 0, 8),  # rows longer than a window
             (gen.banded_uniform(90000, 4, 40000, seed=2), 1, 0, 5),   # beyond 16 bits: form 1
             (gen.power_law(30000, seed=17), 4, 2, 18),
             (gen.laplacian_2d5(37, 29), 1, 0, 12)]
    for A, P, r, seed in cases:
        x = gen.x_normal(A.n_cols, seed)
        ref = oracle.share_reference(A, P, r, x)
        split = oracle.split(A, P, r)
        tune = {"kernel_local": 2, "kernel_remote": 2, "chunk_local": chunk,
                "chunk_remote": chunk, "width": width, "lanes_local": lanes}
        ops, smap = sp.spmv_plan_space_get(P, 2, 7) if P > 1 else (None, None)
        res, _ = run_share(A, P, r, x, ops, smap, tune={**tune, "form": 4}, ref=ref)
        assert_share_parity(res, ref)
        assert res["info"]["form_local"] == _expected_form(split, 4), (A.n_rows, P, r)
        one, _ = run_share(A, P, r, x, ops, smap, tune={**tune, "form": 1}, ref=ref)
        assert one["info"]["form_local"] == 1
        assert np.array_equal(bits(res["y"]), bits(one["y"]))
    for A, P, r in [(gen.laplacian_3d7(32), 4, 1), (gen.stencil_3d27(20, seed=3), 2, 1)]:
        x = gen.x_integer(A.n_cols, 9)
        res, ref = run_share(A, P, r, x, tune={"kernel_local": 2, "form": 4})
        assert res["info"]["form_local"] == 4
        if A.n_rows == 32 ** 3:
            assert np.array_equal(bits(res["y"]), bits(ref["y"]))
        else:
            assert_share_parity(res, ref)


def _dense_remote_rows(n=40000, dense=(20000, 20001, 29999), seed=4):
    """A diagonal matrix whose listed rows also hold every column of the
    first half: on two ranks those rows carry 20,000 remote entries, 2,500
    in each column slab (longer than any window)."""
    rng = np.random.default_rng(seed)
    cols, ptr = [], [0]
    for i in range(n):
        c = np.arange(n // 2, dtype=np.int32) if i in dense else np.empty(0, np.int32)
        c = np.union1d(c, [i]).astype(np.int32)
        cols.append(c)
        ptr.append(ptr[-1] + c.size)
    col = np.concatenate(cols)
    return gen.CSR(n, n, np.asarray(ptr, np.int32), col, rng.standard_normal(col.size))


@pytest.mark.parametrize("chunk,width,lanes,rows", [(0, 0, 0, 0), (4, 2, 1, 1), (8, 4, 2, 1),
                                                    (16, 2, 4, 1), (4, 2, 1, 2), (8, 4, 0, 4),
                                                    (16, 2, 1, 8), (16, 4, 0, 2)])
def test_column_slab_form(chunk, width, lanes, rows):
    """y_R in column slabs (form 5), in tiles of 256 / lanes rows and in
    wide tiles (rows per thread > 1), against the oracle on power-law,
    stencil and banded shares and on rows far longer than a window; every
    plan gives the same bits, whether y_R adds into y itself or a combine
    step adds its partial sums; integer data are exact."""
    log(f"column slabs chunk={chunk} width={width} lanes={lanes} rows={rows}")
    cases = [(gen.power_law(60000, seed=21), 4, 2, 31),
             (gen.power_law(30000, seed=17), 16, 5, 32),
             (gen.stencil_3d27(30, seed=5), 4, 2, 33),
             (gen.banded_random(50000, seed=9), 3, 1, 34),
             (_dense_remote_rows(), 2, 1, 35),
             (gen.laplacian_2d5(37, 29), 3, 2, 36),
             (gen.laplacian_2d5(5, 4), 2, 1, 37)]   # a 5-entry halo: slabs 5-7 empty
    tune = {"kernel_remote": 2, "chunk_remote": chunk, "width": width, "lanes_remote": lanes,
            "rows_remote": rows, "form": 5}
    for A, P, r, seed in cases:
        x = gen.x_normal(A.n_cols, seed)
        ref = oracle.share_reference(A, P, r, x)
        ys, fused = [], set()
        for idx in (7, 468, 1190, 2003):
            ops, smap = sp.spmv_plan_space_get(P, 2, idx)
            res, _ = run_share(A, P, r, x, ops, smap, tune=tune, ref=ref)
            assert res["info"]["form_remote"] == 5, (A.n_rows, P, r)
            assert_share_parity(res, ref)
            ys.append(bits(res["y"]))
            fused.add(res["info"]["fused_combine"])
        assert fused == {0, 1}
        for y in ys[1:]:
            assert np.array_equal(ys[0], y)
        # the explicit Unpack kernel (the default reads the receive buffer
        # in place), and the fine-grained program: the same bits
        fu, _ = run_share(A, P, r, x, tune={**tune, "fuse_unpack": 2}, ref=ref)
        assert fu["info"]["form_remote"] == 5 and np.array_equal(ys[0], bits(fu["y"]))
        plan = sp.spmv_plan_create(A, P, r, None, None, 2, tune)
        try:
            sp.spmv_plan_set_fine(plan)
            fi, _ = run_share(A, P, r, x, ref=ref, plan=plan)
            assert fi["info"]["fine"] == 1 and np.array_equal(ys[0], bits(fi["y"]))
        finally:
            sp.spmv_plan_destroy(plan)
    A = gen.laplacian_3d7(32)   # integer entries: every sum exact
    res, ref = run_share(A, 4, 2, gen.x_integer(A.n_cols, 9), tune=tune)
    assert res["info"]["form_remote"] == 5
    assert np.array_equal(bits(res["y"]), bits(ref["y"]))


@pytest.mark.parametrize("chunk", [0, 8, 16])
def test_sliced16_form(chunk):
    """Sliced ELL with 16-bit row-relative columns against the oracle, and
    bit for bit against the 32-bit sliced form (same entry order): stencils,
    a ragged last slice, offsets close to the 16-bit limit, and the fall
    back to 32-bit columns when offsets exceed it or slices differ in
    width."""
    log(f"sliced16 form chunk={chunk}")
    cases = [(gen.laplacian_3d7(48), 4, 1, 3),
             (gen.stencil_3d27(40, seed=5), 4, 1, 6),
             (gen.laplacian_2d5(37, 29), 1, 0, 12),               # 1073 rows: ragged last slice
             (gen.banded_uniform(90000, 4, 30000, seed=2), 1, 0, 4),   # offsets up to 30,000
             (gen.banded_uniform(90000, 4, 40000, seed=2), 1, 0, 5),   # beyond 16 bits: form 2
             (gen.stencil_3d27(20, seed=3), 4, 1, 7),              # uneven widths: form 2
             (gen.banded_uniform(60000, 10, 15000, seed=8), 4, 3, 9)]
    for A, P, r, seed in cases:
        x = gen.x_normal(A.n_cols, seed)
        ref = oracle.share_reference(A, P, r, x)
        split = oracle.split(A, P, r)
        tune = {"kernel_local": 2, "kernel_remote": 2, "chunk_local": chunk,
                "chunk_remote": chunk}
        ops, smap = sp.spmv_plan_space_get(P, 2, 5) if P > 1 else (None, None)
        res, _ = run_share(A, P, r, x, ops, smap, tune={**tune, "form": 3}, ref=ref)
        assert_share_parity(res, ref)
        assert res["info"]["form_local"] == _expected_form(split, 3), (A.n_rows, P, r)
        two, _ = run_share(A, P, r, x, ops, smap, tune={**tune, "form": 2}, ref=ref)
        assert two["info"]["form_local"] in (1, 2)
        if two["info"]["form_local"] == 2:
            assert np.array_equal(bits(res["y"]), bits(two["y"]))
    for A, P, r in [(gen.laplacian_3d7(32), 4, 1), (gen.laplacian_2d5(64), 1, 0)]:
        x = gen.x_integer(A.n_cols, 9)
        res, ref = run_share(A, P, r, x, tune={"kernel_local": 2, "chunk_local": chunk, "form": 3})
        assert res["info"]["form_local"] == 3
        assert np.array_equal(bits(res["y"]), bits(ref["y"]))


def test_sixteen_bit_boundary():
    """Offsets of exactly +-32767 from the row in the 16-bit sliced form, and
    of +-32512 (plus up to 255 rows within a tile) in 16-bit packed tiles:
    oracle parity and the bits of the 32-bit forms; +-32768 falls back."""
    for d, form, other, expect in ((32767, 3, 2, 3), (32768, 3, 2, 2),
                                   (32767 - 255, 4, 1, 4), (32768, 4, 1, 1)):
        A = gen.three_diagonals(200000, d, seed=d)
        x = gen.x_normal(A.n_cols, 5)
        log(f"16-bit boundary d={d} form={form}")
        res, ref = run_share(A, 1, 0, x, tune={"kernel_local": 2, "form": form})
        assert res["info"]["form_local"] == expect
        assert_share_parity(res, ref)
        base, _ = run_share(A, 1, 0, x, tune={"kernel_local": 2, "form": other}, ref=ref)
        assert np.array_equal(bits(res["y"]), bits(base["y"]))


def test_automatic_form_rule():
    """The automatic choice follows the host rule on every parity case."""
    for A, P, r in [(gen.laplacian_3d7(32), 4, 1), (gen.stencil_3d27(40, seed=5), 4, 1),
                    (gen.banded_uniform(90000, 4, 40000, seed=2), 1, 0),
                    (gen.power_law(30000, seed=17), 4, 2), (gen.power_law(200000, seed=3), 2, 1)]:
        x = gen.x_normal(A.n_cols, 1)
        res, ref = run_share(A, P, r, x)
        assert_share_parity(res, ref)
        assert res["info"]["form_local"] == _expected_form(oracle.split(A, P, r), 0)


def test_sliced_form_all_plans_identical_and_not_batched():
    import torch
    A = gen.stencil_3d27(24, seed=7)
    x = gen.x_normal(A.n_cols, 70)
    P, r = 4, 2
    ref = oracle.share_reference(A, P, r, x)
    first = None
    for i in range(0, 2016, 97):
        ops, smap = sp.spmv_plan_space_get(P, 2, i)
        res, _ = run_share(A, P, r, x, ops, smap, tune={"form": 2}, ref=ref)
        assert res["info"]["form_local"] == 2
        if first is None:
            assert_share_parity(res, ref)
            first = bits(res["y"])
        assert np.array_equal(bits(res["y"]), first), i
    plan = sp.spmv_plan_create(A, P, r, None, None, 2, {"form": 2})
    try:
        with pytest.raises(sp.SpmvError):
            sp.spmv_batch_create([plan])
    finally:
        sp.spmv_plan_destroy(plan)
    torch.cuda.synchronize()


def test_stream_stencils_bit_exact_integer():
    for A, P, r in [(gen.laplacian_3d7(32), 4, 1), (gen.laplacian_2d5(64), 1, 0)]:
        x = gen.x_integer(A.n_cols, 9)
        res, ref = run_share(A, P, r, x, tune={"kernel_local": 2, "kernel_remote": 2})
        assert np.array_equal(bits(res["y"]), bits(ref["y"]))


def test_op_launch_matches_exec():
    """The op-level entry point (used for kernel timing) computes what the
    exec computes: y_L then y_R on one stream."""
    import torch
    A = gen.stencil_3d27(20, seed=3)
    x = gen.x_normal(A.n_cols, 30)
    res, ref = run_share(A, 4, 1, x, keep_plan=True)
    plan = res.pop("plan")
    try:
        info = res["info"]
        lo, n = info["lo"], info["n_loc"]
        xd = torch.from_numpy(x[lo:lo + n].copy()).cuda()
        yd = torch.empty(n, dtype=torch.float64, device="cuda")
        s = torch.cuda.current_stream()
        sp.spmv_op_launch(plan, sp.SPMV_OP_UNPACK, None, None, s)
        sp.spmv_op_launch(plan, sp.SPMV_OP_YL, xd, yd, s)
        sp.spmv_op_launch(plan, sp.SPMV_OP_YR, xd, yd, s)
        torch.cuda.synchronize()
        assert np.array_equal(bits(yd.cpu().numpy()), bits(res["y"]))
        with pytest.raises(sp.SpmvError):
            sp.spmv_op_launch(plan, sp.SPMV_OP_POST_SEND, xd, yd, s)
    finally:
        sp.spmv_plan_destroy(plan)


def test_every_plan_bit_identical():
    """All 2016 plans of the design space give the same y bits (missing
    synchronisation or a race would break this) and pass parity."""
    A = gen.banded_uniform(6000, 10, 1500, seed=21)
    x = gen.x_normal(A.n_cols, 22)
    P, r = 4, 1
    ref = oracle.share_reference(A, P, r, x)
    n = sp.spmv_plan_space_count(P, 2)
    assert n == 2016
    first = None
    fused = 0
    for i in range(n):
        if i % 500 == 0:
            log(f"plan {i}/{n}")
        ops, smap = sp.spmv_plan_space_get(P, 2, i)
        res, _ = run_share(A, P, r, x, ops, smap, 2, ref=ref)
        fused += res["info"]["fused_combine"]
        if first is None:
            assert_share_parity(res, ref)
            first = bits(res["y"])
        else:
            assert np.array_equal(bits(res["y"]), first), i
            assert np.array_equal(bits(res["outbox"]), bits(ref["sendbuf"])), i
        if i % 16 == 0:
            # every 16th plan again with the explicit Unpack kernel
            ex, _ = run_share(A, P, r, x, ops, smap, 2, ref=ref, tune={"fuse_unpack": 2})
            assert ex["info"]["fuse_unpack"] == 0
            assert np.array_equal(bits(ex["y"]), first), i
    assert res["info"]["fuse_unpack"] == 1   # the default reads the receive buffer in place
    assert 0 < fused < n   # both the fused and the combine path were exercised


def test_reorder_and_plan_time():
    """One plan re-ordered through part of the design space keeps giving the
    same bits; the paper's timing protocol returns sane per-sample times."""
    import torch
    A = gen.banded_uniform(8000, 10, 2000, seed=23)
    x = gen.x_normal(A.n_cols, 24)
    P, r = 4, 2
    ref = oracle.share_reference(A, P, r, x)
    ops, smap = sp.spmv_plan_space_get(P, 2, 0)
    plan = sp.spmv_plan_create(A, P, r, ops, smap, 2)
    try:
        first = None
        rng = np.random.default_rng(3)
        for i in rng.choice(2016, 40, replace=False):
            ops, smap = sp.spmv_plan_space_get(P, 2, int(i))
            sp.spmv_plan_reorder(plan, ops, smap, 2)
            res, _ = run_share(A, P, r, x, ref=ref, plan=plan)
            if first is None:
                assert_share_parity(res, ref)
                first = bits(res["y"])
            assert np.array_equal(bits(res["y"]), first), i
        info = sp.spmv_plan_info(plan)
        lo, n = info["lo"], info["n_loc"]
        xd = torch.from_numpy(x[lo:lo + n].copy()).cuda()
        yd = torch.empty(n, dtype=torch.float64, device="cuda")
        t = sp.spmv_plan_time(plan, xd, yd, torch.cuda.current_stream(), 0.005, 3)
        assert t.shape == (3,) and np.all(t > 0) and np.all(t < 0.005)
        # an order needing a third stream does not fit a two-stream plan
        bad = {sp.SPMV_OP_PACK: 0, sp.SPMV_OP_YL: 1, sp.SPMV_OP_YR: 2}
        with pytest.raises(sp.SpmvError) as e:
            sp.spmv_plan_reorder(plan, ops, bad, 3)
        assert e.value.code == sp.SPMV_EPLAN
    finally:
        sp.spmv_plan_destroy(plan)


def test_three_streams_and_explicit_unpack():
    A = gen.banded_uniform(4000, 10, 1000, seed=5)
    x = gen.x_normal(A.n_cols, 6)
    ref = oracle.share_reference(A, 4, 2, x)
    O = sp
    ops = [O.SPMV_OP_START, O.SPMV_OP_POST_RECV, O.SPMV_OP_PACK, O.SPMV_CER_AFTER(O.SPMV_OP_PACK),
           O.SPMV_OP_YL, O.SPMV_CES_B4(O.SPMV_OP_POST_SEND), O.SPMV_OP_POST_SEND,
           O.SPMV_OP_WAIT_RECV, O.SPMV_OP_UNPACK, O.SPMV_CER_AFTER(O.SPMV_OP_UNPACK),
           O.SPMV_CSWE_B4(O.SPMV_OP_YR), O.SPMV_OP_YR, O.SPMV_OP_WAIT_SEND, O.SPMV_OP_END]
    smap = {O.SPMV_OP_PACK: 0, O.SPMV_OP_YL: 1, O.SPMV_OP_UNPACK: 2, O.SPMV_OP_YR: 0}
    res, _ = run_share(A, 4, 2, x, ops, smap, 3, ref=ref, tune={"fuse_unpack": 2})
    assert res["info"]["n_streams"] == 3 and res["info"]["fused_combine"] == 0
    assert res["info"]["fuse_unpack"] == 0
    assert_share_parity(res, ref)
    # the same order with Unpack fused (the default): no kernel, same bits
    fu, _ = run_share(A, 4, 2, x, ops, smap, 3, ref=ref)
    assert fu["info"]["fuse_unpack"] == 1
    assert np.array_equal(bits(fu["y"]), bits(res["y"]))


def test_repeated_exec_new_x():
    """A is static, x is not: one plan, several x vectors."""
    A = gen.banded_uniform(5000, 10, 1250, seed=31)
    plan = sp.spmv_plan_create(A, 4, 1)
    try:
        for s in range(4):
            x = gen.x_normal(A.n_cols, 100 + s)
            res, ref = run_share(A, 4, 1, x, plan=plan)
            assert_share_parity(res, ref)
    finally:
        sp.spmv_plan_destroy(plan)


def test_local_plan_power_law_share():
    """Rank-local plans (own rows + send lists) against the oracle's
    rank-local definition, power-law share of 400k rows, rank 5 of 16."""
    import torch
    d = gen.power_law_share(400_000, 16, 5, seed=4001)
    x = gen.x_normal(d["n_global"], 4101)
    ref = oracle.share_reference_local(d["local"], d["n_global"], 16, 5, d["send_idx"],
                                       d["send_off"], x)
    for tune in ({}, {"kernel_local": 1, "kernel_remote": 1}):
        plan = sp.spmv_plan_create_local(d["local"], d["n_global"], 16, 5, d["send_idx"],
                                         d["send_off"], tune=tune)
        try:
            res, _ = run_share(None, 16, 5, x, ref=ref, plan=plan)
            assert_share_parity(res, ref)
        finally:
            sp.spmv_plan_destroy(plan)


# ------------------------------------------------------------ edge cases

def test_empty_share_and_empty_rows():
    A = gen.laplacian_2d5(2, 2)               # 4 rows over 6 ranks
    x = gen.x_normal(4, 1)
    for r in range(6):
        res, ref = run_share(A, 6, r, x)
        assert_share_parity(res, ref)
    # matrix with empty rows and a block-diagonal rank (no halo at all)
    rp = np.array([0, 0, 2, 2, 3, 3, 5, 5], np.int32)
    ci = np.array([0, 1, 3, 5, 6], np.int32)
    B = gen.CSR(7, 7, rp, ci, np.array([1.5, -2.0, 3.0, 0.25, 7.0]))
    x = gen.x_normal(7, 2)
    for P in (1, 2, 3):
        for r in range(P):
            res, ref = run_share(B, P, r, x)
            assert_share_parity(res, ref)
    # every entry remote: empty local blocks over owned rows, in every form
    n = 256
    rows = np.arange(n)
    C = gen.CSR(n, n, np.arange(n + 1, dtype=np.int32), ((rows + n // 2) % n).astype(np.int32),
                np.linspace(-1.0, 1.0, n))
    x = gen.x_normal(n, 3)
    for form in (0, 1, 2, 3, 4, 5):
        res, ref = run_share(C, 2, 1, x, tune={"kernel_local": 2, "form": form})
        assert res["info"]["nnz_local"] == 0
        assert_share_parity(res, ref)
    assert res["info"]["form_remote"] == 5


def check_tuner_choice(best, res, cands, margin=0.02):
    assert [d["tune"] for d in res] == [{}] + list(cands)
    assert all(d["us"] > 0 for d in res)
    fastest = min(res, key=lambda d: d["us"])
    if fastest["us"] <= res[0]["us"] * (1 - margin):
        assert best == fastest["tune"]
    else:
        assert best == {}


def test_kernel_autotuner():
    """The kernel autotuner times the automatic choice and every candidate
    and returns the fastest, keeping the automatic choice unless a
    candidate beats it by more than the margin; the tune it returns
    computes y within tolerance."""
    from paper_2203_02530_amd import tune as tuner
    A = gen.laplacian_3d7(48)
    P, r = 4, 1
    x = gen.x_normal(A.n_cols, 81)
    cands = [{"kernel_local": 2, "form": 3, "chunk_local": 8},
             {"kernel_local": 2, "form": 2, "chunk_local": 8},
             {"kernel_local": 2, "form": 4, "chunk_local": 4, "width": 2},
             {"kernel_local": 2, "form": 1, "chunk_local": 4, "width": 2},
             {"kernel_local": 1, "lanes_local": 8, "rows_local": 4}]
    best, res = tuner.tune_kernel(A, P, r, x, candidates=cands, launches=20)
    check_tuner_choice(best, res, cands)
    out, ref = run_share(A, P, r, x, tune=best)
    assert_share_parity(out, ref)


def test_remote_autotuner():
    """The same search over y_R's forms (packed tiles with 1, 2, 4 lanes,
    sliced, column slabs with 1, 2 lanes) on a power-law share whose halo
    is larger than one XCD's L2: every candidate timed, the fastest
    returned, its plan within tolerance of the oracle."""
    from paper_2203_02530_amd import tune as tuner
    A = gen.power_law(1_000_000, seed=44)
    P, r = 8, 3
    x = gen.x_normal(A.n_cols, 82)
    cands = list(tuner.DEFAULT_REMOTE_CANDIDATES)
    best, res = tuner.tune_kernel(A, P, r, x, candidates=cands, launches=20, op=sp.SPMV_OP_YR)
    check_tuner_choice(best, res, cands)
    log("remote autotuner: " + ", ".join(f'{d["tune"].get("form", "auto")}/{d["tune"].get("lanes_remote", 0)}'
                                          f' {d["us"]:.1f} us' for d in res))
    out, ref = run_share(A, P, r, x, tune=best)
    assert_share_parity(out, ref)
    with pytest.raises(ValueError):
        tuner.tune_kernel(A, P, r, x, candidates=cands[:1], op=sp.SPMV_OP_PACK)


@pytest.mark.parametrize("plan_index", [332, 1500, 71, 1190, 2003])
def test_exec_orders_after_pending_caller_work(plan_index):
    """The exec runs after work still pending on the caller's stream (its
    plan stream 0 is that stream; other plan streams wait at start) and
    returns with y complete: x is written by an asynchronous copy on a side
    stream just before the exec, y read without a further synchronisation."""
    import torch
    A = gen.laplacian_3d7(48)
    P, r = 4, 1
    x = gen.x_normal(A.n_cols, 77)
    ref = oracle.share_reference(A, P, r, x)
    ops, smap = sp.spmv_plan_space_get(P, 2, plan_index)
    plan = sp.spmv_plan_create(A, P, r, ops, smap, 2)
    try:
        info = sp.spmv_plan_info(plan)
        lo, n = info["lo"], info["n_loc"]
        sp.spmv_plan_inbox(plan)[:] = ref["inbox"]
        src = torch.from_numpy(np.ascontiguousarray(x[lo:lo + n])).cuda()
        big = torch.empty(1 << 26, dtype=torch.float64, device="cuda")
        xd = torch.zeros(n, dtype=torch.float64, device="cuda")
        yd = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
        side = torch.cuda.Stream()
        torch.cuda.synchronize()
        with torch.cuda.stream(side):
            for _ in range(4):
                big.mul_(1.0)               # ~2 GB of traffic queued ahead of x
            xd.copy_(src)
            sp.spmv_exec(plan, xd, yd, side)
            y = yd.cpu().numpy()            # no synchronisation in between
        assert info["n_streams"] >= 1
        ok = oracle.within_tolerance(y, ref["y"], ref["absax"], 1e-12)
        assert ok.all(), np.flatnonzero(~ok)[:10]
    finally:
        sp.spmv_plan_destroy(plan)


def test_long_rows():
    """Rows far longer than a wavefront (up to 10^4 entries)."""
    A = gen.power_law(40000, mean_len=200.0, sigma=1.2, max_len=10000, seed=44)
    x = gen.x_normal(A.n_cols, 45)
    for kern, lanes in ((0, 0), (1, 64), (1, 8), (2, 16)):
        res, ref = run_share(A, 4, 1, x, tune={"kernel_local": kern, "kernel_remote": kern,
                                               "lanes_local": lanes, "lanes_remote": lanes})
        assert_share_parity(res, ref)


def test_profile_counters():
    A = gen.laplacian_3d7(24)
    x = gen.x_uniform(A.n_cols, 3)
    plan = sp.spmv_plan_create(A, 4, 1, tune={"flags": sp.SPMV_F_PROFILE, "fuse_unpack": 2})
    try:
        for _ in range(3):
            run_share(A, 4, 1, x, plan=plan)
        cnt = sp.spmv_plan_get_f64(plan, sp.SPMV_F64_OP_COUNT)
        ms = sp.spmv_plan_get_f64(plan, sp.SPMV_F64_OP_MS)
        for op in (sp.SPMV_OP_PACK, sp.SPMV_OP_YL, sp.SPMV_OP_UNPACK, sp.SPMV_OP_YR):
            assert cnt[op] == 3 and ms[op] > 0
        sp.spmv_plan_reset_times(plan)
        assert sp.spmv_plan_get_f64(plan, sp.SPMV_F64_OP_COUNT).sum() == 0
        # host timeline: one cumulative mark per token, in order
        sp.spmv_plan_set_profile(plan, False, host=True)
        for _ in range(4):
            res, _ = run_share(A, 4, 1, x, plan=plan)
        assert_share_parity(res, oracle.share_reference(A, 4, 1, x))
        n_ops = sp.spmv_plan_info(plan)["n_ops"]
        hus = sp.spmv_plan_get_f64(plan, sp.SPMV_F64_HOST_US)
        assert hus.size == n_ops
        assert sp.spmv_plan_get_f64(plan, sp.SPMV_F64_HOST_COUNT)[0] == 4
        assert np.all(hus > 0) and np.all(np.diff(hus) >= 0)
        assert sp.spmv_plan_get_f64(plan, sp.SPMV_F64_OP_COUNT).sum() == 0   # events off
        ops, smap = sp.spmv_plan_space_get(4, 2, 9)
        sp.spmv_plan_reorder(plan, ops, smap, 2)                               # clears it
        assert sp.spmv_plan_get_f64(plan, sp.SPMV_F64_HOST_COUNT)[0] == 0
        with pytest.raises(sp.SpmvError):
            sp._check(sp._lib.spmv_plan_set_profile(plan, 4))
    finally:
        sp.spmv_plan_destroy(plan)


# ------------------------------------------------------------ full sizes

def _sampled(res, ref, rows):
    ok = oracle.within_tolerance(res["y"][rows], ref["y"][rows], ref["absax"][rows])
    assert ok.all()


def _resident_bits(res, x, mode):
    """The resident step of the plan in `res` (its receive buffer holds the
    halo of the exec that made `res`): its launch mode, and y's bits equal
    to that exec's, twice in a row."""
    import torch
    plan, info = res["plan"], res["info"]
    assert info["resident_grouped"] == mode
    lo, n = info["lo"], info["n_loc"]
    xd = torch.from_numpy(np.ascontiguousarray(x[lo:lo + n])).cuda()
    for _ in range(2):
        yd = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
        sp.spmv_exec_resident(plan, xd, yd, torch.cuda.current_stream())
        torch.cuda.synchronize()
        assert np.array_equal(bits(yd.cpu().numpy()), bits(res["y"]))


def test_full_laplace3d_128_p4_rank1():
    """The measured workload at full size, in the launch configuration the
    benchmark times, every row checked; its resident step (the whole step
    in y_L's launch) gives the exec's bits."""
    A = gen.laplacian_3d7(128)
    x = gen.x_uniform(A.n_cols, 2)
    log("full 3D 7-point 128^3 P=4 r=1")
    res, ref = run_share(A, 4, 1, x, keep_plan=True)
    try:
        info = res["info"]
        assert info["n_loc"] == 524288 and info["nnz_local"] == 3620864
        assert info["n_halo"] == 32768 and info["n_send"] == 32768
        assert_share_parity(res, ref)
        _resident_bits(res, x, 3)
    finally:
        sp.spmv_plan_destroy(res["plan"])


def test_full_stencil27_150_p8_rank3():
    """As above for the 27-point share (its resident step: Pack in y_L's
    launch, then y_R)."""
    A = gen.stencil_3d27(150, seed=3)
    x = gen.x_normal(A.n_cols, 30)
    log("full 3D 27-point 150^3 P=8 r=3")
    res, ref = run_share(A, 8, 3, x, keep_plan=True)
    try:
        info = res["info"]
        assert info["n_loc"] == 421875 and info["n_halo"] == 45151
        assert_share_parity(res, ref)
        _resident_bits(res, x, 3)
    finally:
        sp.spmv_plan_destroy(res["plan"])


@pytest.mark.parametrize("tune", [
    {"kernel_local": 2, "kernel_remote": 2, "chunk_local": 8, "chunk_remote": 8, "width": 2,
     "form": 1},
    {"kernel_local": 2, "kernel_remote": 2, "chunk_local": 4, "chunk_remote": 4, "width": 2,
     "form": 5}])
def test_full_powerlaw_4m_p16_rank5_and_batch(tune):
    """The power-law 4M-row share (rank 5 of 16) at full size against the
    oracle's rank-local definition, every row checked, alone and in a batch
    of two full shares (bit-identical to the solo execs), with y_R in packed
    tiles and in column slabs (the variant the batch autotuner picks for
    the benchmark's 64-share batch), in the automatic batch options and in
    persistent blocks."""
    import torch
    shares, plans, refs, xs, ys = [], [], [], [], []
    try:
        for seed in (4000, 4001):
            log(f"full power-law 4M share seed {seed}")
            d = gen.power_law_share(4_000_000, 16, 5, seed=seed)
            x = gen.x_normal(d["n_global"], seed + 100)
            ref = oracle.share_reference_local(d["local"], d["n_global"], 16, 5, d["send_idx"],
                                               d["send_off"], x)
            plan = sp.spmv_plan_create_local(d["local"], d["n_global"], 16, 5, d["send_idx"],
                                             d["send_off"], tune=tune)
            plans.append(plan)
            res, _ = run_share(None, 16, 5, x, ref=ref, plan=plan)
            assert res["info"]["n_loc"] == 250_000
            assert res["info"]["form_remote"] == tune["form"]
            assert_share_parity(res, ref)
            info = res["info"]
            lo, n = info["lo"], info["n_loc"]
            xs.append(torch.from_numpy(np.ascontiguousarray(x[lo:lo + n])).cuda())
            ys.append(torch.full((n,), float("nan"), dtype=torch.float64, device="cuda"))
            refs.append(res["y"])
        for opts in ({}, {"persistent": 1}):
            for y in ys:
                y.fill_(float("nan"))
            b = sp.spmv_batch_create(plans, opts)
            try:
                sp.spmv_batch_exec(b, xs, ys, torch.cuda.current_stream())
                for y, solo in zip(ys, refs):
                    assert np.array_equal(bits(y.cpu().numpy()), bits(solo)), opts
            finally:
                sp.spmv_batch_destroy(b)
    finally:
        for p in plans:
            sp.spmv_plan_destroy(p)


def test_full_powerlaw_4m_global_p16_rank5_column_slabs():
    """Rank 5's share of the global 4M-row power-law matrix (16 ranks, the
    whole matrix generated, so the send lists and the halo come from the
    real partition), in the launch configuration the benchmark times: the
    automatic form puts y_R in column slabs (its 19 MB halo exceeds one
    XCD's L2).  Every row against the oracle, the outbox and
    receive buffer bit-exact, then 8 plans spread over the space on the same
    uploaded share, each bit-identical to the first; the resident step the
    benchmark times (two grouped launches, and each launch alone) gives the
    same bits on the halo that exec left in the receive buffer; wide slab
    tiles (rows_remote = 4) agree with the oracle too."""
    import torch
    w = gen.WORKLOADS["powerlaw_4m_p16r5"]
    A = w["build"]()
    x = w["x"](A.n_cols)
    P, r = w["nranks"], w["rank"]
    log("full global power-law 4M P=16 r=5, automatic form")
    ref = oracle.share_reference(A, P, r, x)
    res, _ = run_share(A, P, r, x, ref=ref, keep_plan=True)
    plan = res.pop("plan")
    try:
        info = res["info"]
        assert info["n_loc"] == 250_000 and info["form_remote"] == 5
        assert info["rows_remote"] == 1 and info["lanes_remote"] == 1
        assert info["n_halo"] * 8 > 4 << 20
        assert_share_parity(res, ref)
        first = bits(res["y"])
        n = sp.spmv_plan_space_count(P, 2)
        for i in np.linspace(0, n - 1, 8).astype(int):
            ops, smap = sp.spmv_plan_space_get(P, 2, int(i))
            sp.spmv_plan_reorder(plan, ops, smap, 2)
            got, _ = run_share(A, P, r, x, ref=ref, plan=plan)
            assert np.array_equal(bits(got["y"]), first), i
        assert info["resident_grouped"] == 1
        lo, n_loc = info["lo"], info["n_loc"]
        xd = torch.from_numpy(np.ascontiguousarray(x[lo:lo + n_loc])).cuda()
        yd = torch.full((n_loc,), float("nan"), dtype=torch.float64, device="cuda")
        s = torch.cuda.current_stream()
        for _ in range(3):
            sp.spmv_exec_resident(plan, xd, yd, s)
        torch.cuda.synchronize()
        assert np.array_equal(bits(yd.cpu().numpy()), first)
        assert np.array_equal(bits(sp.spmv_plan_get_f64(plan, sp.SPMV_F64_SENDBUF)),
                              bits(ref["sendbuf"]))
        yd.fill_(float("nan"))
        sp.spmv_exec_resident_part(plan, 0, xd, yd, s)
        sp.spmv_exec_resident_part(plan, 1, xd, yd, s)
        torch.cuda.synchronize()
        assert np.array_equal(bits(yd.cpu().numpy()), first)
    finally:
        sp.spmv_plan_destroy(plan)
    log("full global power-law 4M P=16 r=5, wide slab tiles")
    res, _ = run_share(A, P, r, x, ref=ref, tune={"form": 5, "rows_remote": 4})
    assert res["info"]["form_remote"] == 5 and res["info"]["rows_remote"] == 4
    assert_share_parity(res, ref)


def test_full_paper_banded_150k_p4_rank1_sampled_plans():
    """The paper's own input at full size (Sec. III: 150,000 rows, 10
    entries per row in half-bandwidth 37,500, P = 4; rank 1), in the launch
    configuration the benchmark times: the default plan against the oracle
    on every row, then 24 plans spread over the space on the same uploaded
    share (re-ordered in place), each bit-identical to the first and with an
    exact outbox.  Its column offsets exceed 16 bits, so y_L runs packed tiles
    with 32-bit columns here (the 6,000-row all-plans case runs another
    form)."""
    A = gen.banded_uniform(150_000, 10, 37_500, seed=100)
    x = gen.x_normal(A.n_cols, 101)
    P, r = 4, 1
    log("full banded 150k P=4 r=1")
    ref = oracle.share_reference(A, P, r, x)
    res, _ = run_share(A, P, r, x, ref=ref, keep_plan=True)
    plan = res.pop("plan")
    try:
        info = res["info"]
        assert info["n_loc"] == 37_500 and info["form_local"] == 1
        assert info["nnz_local"] + info["nnz_remote"] == 375_000
        assert_share_parity(res, ref)
        first = bits(res["y"])
        n = sp.spmv_plan_space_count(P, 2)
        for i in np.linspace(0, n - 1, 24).astype(int):
            ops, smap = sp.spmv_plan_space_get(P, 2, int(i))
            sp.spmv_plan_reorder(plan, ops, smap, 2)
            got, _ = run_share(A, P, r, x, ref=ref, plan=plan)
            assert np.array_equal(bits(got["y"]), first), i
            assert np.array_equal(bits(got["outbox"]), bits(ref["sendbuf"])), i
    finally:
        sp.spmv_plan_destroy(plan)


def _two_remote_per_row(n_half=4096, seed=0, uneven_local=False):
    """Two ranks; rank 0's rows hold their diagonal (and with uneven_local
    0-2 more local entries, so that y_L's slices differ in width) and
    exactly two entries in rank 1's block (so its remote rows are one
    uniform sliced width of 2), rank 1's rows their diagonal only."""
    rng = np.random.default_rng(seed)
    ptr, cols = [0], []
    for i in range(2 * n_half):
        c = [i]
        if i < n_half:
            c += [n_half + (7 * i) % n_half, n_half + (7 * i + 13) % n_half]
            if uneven_local:
                c += [(i + 1 + k * 97) % n_half for k in range(i % 3)]
        c = sorted(set(c))
        cols.append(np.asarray(c, np.int32))
        ptr.append(ptr[-1] + len(c))
    col = np.concatenate(cols)
    return gen.CSR(2 * n_half, 2 * n_half, np.asarray(ptr, np.int32), col,
                   rng.standard_normal(col.size))


def _long_local_rows(n_half=6000, seed=0):
    """Two ranks; rank 0's rows hold a local band of three, a few of them
    3,000 or more local entries (longer than a packed window), and every
    seventh row and the long rows 5 and 5,999 one to five entries in rank
    1's block; rank 1's rows their diagonal.  So y_R is in packed tiles
    with one summing lane, and some of y_L's single-row tiles have remote
    entries."""
    rng = np.random.default_rng(seed)
    long_rows = {5, 700, 2999, 5990, n_half - 1}
    ptr, cols = [0], []
    for i in range(2 * n_half):
        c = {i}
        if i < n_half:
            c |= {max(i - 1, 0), min(i + 1, n_half - 1)}
            if i in long_rows:
                c |= set(range(0, 3000 + i % 7))
            if i % 7 == 3 or i in (5, n_half - 1):
                c |= {n_half + int(v) for v in rng.integers(0, n_half, 1 + i % 5)}
        c = sorted(c)
        cols.append(np.asarray(c, np.int32))
        ptr.append(ptr[-1] + len(c))
    col = np.concatenate(cols)
    return gen.CSR(2 * n_half, 2 * n_half, np.asarray(ptr, np.int32), col,
                   rng.standard_normal(col.size))


def _remote_per_row(n_remote, n_half=4096, seed=0):
    """Two ranks; rank 0's rows hold 4 local entries and n_remote in rank
    1's block, rank 1's rows their diagonal and one entry in rank 0's block
    (so rank 0 has a send list): in packed tiles of 1,024 entries (256
    rows) a tile's rows hold 256 * n_remote remote entries, exactly a
    window's worth with 4."""
    rng = np.random.default_rng(seed)
    ptr, cols = [0], []
    for i in range(2 * n_half):
        if i < n_half:
            c = [(i + k) % n_half for k in range(4)]
            c += [n_half + (i * 13 + k * 1031) % n_half for k in range(n_remote)]
        else:
            c = [i - n_half, i]
        c = sorted(set(c))
        cols.append(np.asarray(c, np.int32))
        ptr.append(ptr[-1] + len(c))
    col = np.concatenate(cols)
    return gen.CSR(2 * n_half, 2 * n_half, np.asarray(ptr, np.int32), col,
                   rng.standard_normal(col.size))


@pytest.mark.parametrize("mode", ["grouped", "sequential"])
def test_exec_resident_matches_exec(mode):
    """The device work alone (halo already in the receive buffer): the bits
    of spmv_exec for the same halo, the send buffer exact, and no copy from
    the inbox (a changed inbox does not reach y until the next spmv_exec).
    Two grouped launches (Pack, y_L and the column-slab tiles as the items
    of one, the slab sums of the other) where y_R is in column slabs and
    y_L in packed tiles (32- or 16-bit columns) of one window and width,
    with one or two summing lanes and rows longer than a window (mode 1);
    else, where y_L is in packed tiles or the 16-bit sliced form, the whole
    step in y_L's launch, Pack as extra blocks and each row's remote sum
    added where its local sum is stored, when y_R is sliced (an fma chain,
    one or two entries per row) or packed with one summing lane and no row
    longer than a window (mode 3; with both in packed tiles each tile's
    block loads its rows' remote entries, at most a window's worth), or
    Pack alone in y_L's launch and y_R after it (mode 2); otherwise, or
    with the flag, the ops one by one."""
    import torch
    flags = {"grouped": 0, "sequential": sp.SPMV_F_RESIDENT_SEQUENTIAL}[mode]
    long_pl = gen.power_law(40000, mean_len=200.0, sigma=1.2, max_len=10000, seed=44)
    cases = [(gen.power_law(30000, seed=17), 16, 5, 19, {"form": 5}, 1),
             (gen.power_law(60000, seed=21), 8, 3, 22, {"form": 5, "lanes_remote": 2}, 1),
             (gen.power_law(20000, mean_len=100.0, sigma=1.5, max_len=30000, seed=45), 4, 1,
              23, {"form": 5}, 1),                                          # long rows
             (gen.power_law(30000, seed=17), 16, 5, 19, {"form": 5, "width": 4, "chunk_local": 8,
                                                         "chunk_remote": 8}, 1),
             (gen.power_law(30000, seed=17), 4, 2, 18, {}, 2),           # long remote rows
             (gen.power_law(30000, seed=17), 4, 2, 18, {"form": 1}, 2),  # 32-bit y_L columns
             (gen.power_law(30000, seed=17), 4, 2, 18, {"lanes_remote": 2}, 2),
             (gen.power_law(30000, seed=17), 4, 2, 18, {"lanes_remote": 4}, 2),
             (gen.power_law(30000, seed=17), 4, 2, 18, {"form": 1, "chunk_local": 8,
                                                       "chunk_remote": 4}, 2),
             (long_pl, 4, 1, 26, {"form": 1, "lanes_remote": 1}, 2),      # y_R rows beyond a window
             # the whole step in y_L's launch: packed y_L (32-bit, 16-bit
             # columns) or 16-bit sliced y_L, with packed y_R (rounded
             # products) or sliced y_R (fma chains) of at most 4 entries
             (gen.banded_uniform(90000, 4, 30000, seed=2), 4, 1, 27, {"form": 3}, 3),
             (gen.laplacian_3d7(24), 4, 1, 20, {"form": 4}, 3),
             (gen.banded_uniform(60000, 3, 2000, seed=3), 4, 2, 28, {"form": 3}, 3),
             (_two_remote_per_row(), 2, 0, 29, {}, 3),
             (_two_remote_per_row(uneven_local=True), 2, 0, 30, {}, 3),
             (gen.banded_uniform(90000, 6, 2000, seed=3), 4, 2, 28, {"form": 3}, 2),  # 6 entries
             (_dense_remote_rows(), 2, 1, 23, {"form": 5}, 0),            # nothing to send
             (gen.power_law(30000, seed=17), 16, 5, 19, {"form": 5, "fuse_unpack": 2}, 2),
             (gen.power_law(30000, seed=17), 16, 5, 19, {"form": 5, "rows_remote": 2}, 2),
             (gen.power_law(30000, seed=17), 16, 5, 19, {"form": 5, "kernel_local": 1}, 0),
             (gen.power_law(30000, seed=17), 16, 5, 19, {"form": 5, "chunk_local": 8,
                                                         "chunk_remote": 4}, 2),
             (gen.laplacian_3d7(24), 4, 1, 20, {}, 3),                   # 16-bit sliced y_L
             (gen.stencil_3d27(30, seed=5), 4, 2, 24, {}, 3),          # 12 remote entries
             # packed y_L (16-bit, 32-bit, two summing lanes) whose rows
             # longer than a window sum their remote part one by one
             (_long_local_rows(), 2, 0, 31, {}, 3),
             (_long_local_rows(seed=1), 2, 0, 32, {"form": 1}, 3),
             (_long_local_rows(seed=2), 2, 0, 33, {"lanes_local": 2}, 3),
             (_long_local_rows(seed=3), 2, 0, 36, {"lanes_local": 4}, 3),
             (_long_local_rows(seed=4), 2, 0, 37, {"chunk_local": 8, "chunk_remote": 8}, 3),
             (_long_local_rows(seed=5), 2, 0, 38, {"xcd_remap": 2}, 3),   # no XCD ranges
             # a tile's remote entries at the window's 1,024, and past it
             (_remote_per_row(4), 2, 0, 34, {"form": 1}, 3),
             (_remote_per_row(5), 2, 0, 35, {"form": 1}, 2),
             (gen.stencil_3d27(20, seed=3), 4, 1, 25, {"form": 2}, 0),   # 32-bit sliced y_L
             (gen.laplacian_2d5(40), 1, 0, 21, {"form": 1}, 0)]          # one rank
    for A, P, r, seed, tune, grouped in cases:
        tune = {**tune, "flags": flags}
        log(f"exec_resident {mode} n={A.n_rows} P={P} r={r} {tune}")
        x = gen.x_normal(A.n_cols, seed)
        ref = oracle.share_reference(A, P, r, x)
        res, _ = run_share(A, P, r, x, tune=tune, ref=ref, keep_plan=True)
        plan = res.pop("plan")
        try:
            info = res["info"]
            assert info["resident_grouped"] == (grouped if mode != "sequential" else 0), tune
            lo, n = info["lo"], info["n_loc"]
            bufs = sp.spmv_plan_device_buffers(plan)
            assert bufs["n_send"] == info["n_send"] and bufs["n_halo"] == info["n_halo"]
            assert bufs["recv"] != 0 or info["n_halo"] == 0
            xd = torch.from_numpy(np.ascontiguousarray(x[lo:lo + n])).cuda()
            for rep in range(2):
                yd = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
                sp.spmv_exec_resident(plan, xd, yd, torch.cuda.current_stream())
                torch.cuda.synchronize()
                assert np.array_equal(bits(yd.cpu().numpy()), bits(res["y"]))
                if info["resident_grouped"] == 1:   # its two launches one at a time
                    yd.fill_(float("nan"))
                    for part in (0, 1):
                        sp.spmv_exec_resident_part(plan, part, xd, yd,
                                                   torch.cuda.current_stream())
                    torch.cuda.synchronize()
                    assert np.array_equal(bits(yd.cpu().numpy()), bits(res["y"]))
                else:
                    with pytest.raises(sp.SpmvError) as e:
                        sp.spmv_exec_resident_part(plan, 0, xd, yd, torch.cuda.current_stream())
                    assert e.value.code == sp.SPMV_ESTATE
                assert np.array_equal(bits(sp.spmv_plan_get_f64(plan, sp.SPMV_F64_SENDBUF)),
                                      bits(ref["sendbuf"]))
                sp.spmv_plan_inbox(plan)[:] = 0.0     # not copied by the resident exec
        finally:
            sp.spmv_plan_destroy(plan)
