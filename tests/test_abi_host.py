"""Host-side checks of the C-ABI library (no GPU work is launched).

* the shared library loads and exports every function include/spmv.h declares;
* the plan validator and the plan-space enumerator agree with the oracle's
  brute force over permutations (same set of plans, by operation names);
* host-only plans build the rank share bit-exactly like the oracle;
* malformed CSRs and invalid plans return the documented error codes.
"""
import ctypes
import os
import re

import numpy as np
import pytest

import gen
import oracle
import paper_2203_02530_amd as sp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

NAME_OF = {sp.SPMV_OP_START: "start", sp.SPMV_OP_PACK: "Pack", sp.SPMV_OP_YL: "yL",
           sp.SPMV_OP_POST_SEND: "PostSend", sp.SPMV_OP_POST_RECV: "PostRecv",
           sp.SPMV_OP_WAIT_SEND: "WaitSend", sp.SPMV_OP_WAIT_RECV: "WaitRecv",
           sp.SPMV_OP_UNPACK: "Unpack", sp.SPMV_OP_YR: "yR", sp.SPMV_OP_END: "end"}
CODE_OF = {v: k for k, v in NAME_OF.items()}
CODE_OF["CER-after-Pack"] = sp.SPMV_CER_AFTER(sp.SPMV_OP_PACK)
CODE_OF["CES-b4-PostSend"] = sp.SPMV_CES_B4(sp.SPMV_OP_POST_SEND)
HOST_ONLY = {"flags": sp.SPMV_F_HOST_ONLY}


def setup_module(_):
    oracle.build(force=False)


def _header_functions():
    txt = open(os.path.join(ROOT, "include", "spmv.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(spmv_[a-z0-9_]+)\s*\(", txt)) - {
        "spmv_CER_AFTER", "spmv_CES_B4", "spmv_CSWE_B4"})


def test_library_exports_every_declared_function():
    lib = ctypes.CDLL(sp.LIB_PATH)
    names = _header_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n


def test_op_names_match_paper():
    for name, code in CODE_OF.items():
        assert sp.spmv_op_name(code) == name
    with pytest.raises(sp.SpmvError):
        sp.spmv_op_name(0x7f)


# ------------------------------------------------------------ plan space

def _library_space(nranks, S):
    out = set()
    for i in range(sp.spmv_plan_space_count(nranks, S)):
        ops, smap = sp.spmv_plan_space_get(nranks, S, i)
        names = tuple(sp.spmv_op_name(int(o)) for o in ops)
        out.add((names, (int(smap[sp.SPMV_OP_PACK]), int(smap[sp.SPMV_OP_YL]),
                         int(smap[sp.SPMV_OP_YR]))))
    return out


@pytest.mark.parametrize("S", [1, 2, 3])
def test_plan_space_equals_oracle_brute_force(S):
    lib = _library_space(4, S)
    ref = oracle.plan_space(S)
    assert len(lib) == sp.spmv_plan_space_count(4, S)   # no duplicates
    assert lib == ref


def test_plan_space_every_entry_validates():
    for i in range(sp.spmv_plan_space_count(4, 2)):
        ops, smap = sp.spmv_plan_space_get(4, 2, i)
        assert sp.spmv_plan_validate(4, ops, smap, 2) == sp.SPMV_OK


def test_single_rank_space():
    assert sp.spmv_plan_space_count(1, 2) == 1
    ops, smap = sp.spmv_plan_space_get(1, 2, 0)
    assert ops.tolist() == [sp.SPMV_OP_START, sp.SPMV_OP_YL, sp.SPMV_OP_END]


def _codes(names):
    return [CODE_OF[n] for n in names]


def _paper_sequence(numbers):
    """A paper traversal (vertex numbers, Sec. III-A) with the Table III pair
    inserted right before PostSend and Unpack left implied."""
    num = {1: "start", 2: "Pack", 3: "yL", 4: "PostSend", 5: "PostRecv",
           6: "WaitSend", 7: "WaitRecv", 8: "Unpack", 9: "yR", 10: "end"}
    out = []
    for v in numbers:
        name = num[v]
        if name == "Unpack":
            continue
        if name == "PostSend":
            out += ["CER-after-Pack", "CES-b4-PostSend"]
        out.append(name)
    return out


def test_paper_sequences_validate():
    smap = np.full(10, -1, np.int32)
    smap[[sp.SPMV_OP_PACK, sp.SPMV_OP_YL, sp.SPMV_OP_YR]] = [0, 1, 0]
    for seq in ([1, 2, 3, 4, 5, 6, 7, 8, 9, 10], [1, 5, 3, 2, 4, 7, 6, 8, 9, 10]):
        assert sp.spmv_plan_validate(4, _codes(_paper_sequence(seq)), smap, 2) == sp.SPMV_OK


def _swap(o, a, b):
    i, j = o.index(a), o.index(b)
    o[i], o[j] = o[j], o[i]
    return o


BASE = ["start", "PostRecv", "Pack", "CER-after-Pack", "yL", "CES-b4-PostSend",
        "PostSend", "WaitRecv", "yR", "WaitSend", "end"]


@pytest.mark.parametrize("mutate,code", [
    (lambda o: [t for t in o if t != "CES-b4-PostSend"], sp.SPMV_EPLAN),          # missing sync
    (lambda o: [t for t in o if t != "CER-after-Pack"], sp.SPMV_EPLAN),
    (lambda o: o[:1] + ["PostSend"] + [t for t in o[1:] if t != "PostSend"], sp.SPMV_EPLAN),
    (lambda o: ["Pack"] + [t for t in o if t != "Pack"], sp.SPMV_EPLAN),          # start not first
    (lambda o: o[:-1], sp.SPMV_EPLAN),                                               # no end
    (lambda o: o[:2] + ["yL"] + o[2:], sp.SPMV_EPLAN),                               # duplicate
    (lambda o: [t for t in o if t != "WaitRecv"], sp.SPMV_EPLAN),                    # missing vertex
    (lambda o: _swap(o, "WaitRecv", "yR"), sp.SPMV_EPLAN),                          # yR before WaitRecv
    (lambda o: _swap(o, "CER-after-Pack", "CES-b4-PostSend"), sp.SPMV_EPLAN),       # wait before record
])
def test_invalid_plans_rejected(mutate, code):
    smap = np.full(10, -1, np.int32)
    smap[[sp.SPMV_OP_PACK, sp.SPMV_OP_YL, sp.SPMV_OP_YR]] = [0, 1, 1]
    assert sp.spmv_plan_validate(4, _codes(BASE), smap, 2) == sp.SPMV_OK
    assert sp.spmv_plan_validate(4, _codes(mutate(list(BASE))), smap, 2) == code


def test_invalid_tokens_and_streams():
    smap = np.full(10, -1, np.int32)
    smap[[sp.SPMV_OP_PACK, sp.SPMV_OP_YL, sp.SPMV_OP_YR]] = [0, 1, 2]
    assert sp.spmv_plan_validate(4, _codes(BASE), smap, 2) == sp.SPMV_EPLAN    # stream 2 of 2
    bad = _codes(BASE)
    bad.insert(3, 0x7f)
    smap[sp.SPMV_OP_YR] = 1
    assert sp.spmv_plan_validate(4, bad, smap, 2) == sp.SPMV_EPLAN             # unknown token
    extra = _codes(BASE)
    extra.insert(5, sp.SPMV_CER_AFTER(sp.SPMV_OP_YL))
    assert sp.spmv_plan_validate(4, extra, smap, 2) == sp.SPMV_EPLAN           # unneeded sync
    assert sp.spmv_plan_validate(4, _codes(BASE), smap, 0) == sp.SPMV_EINVAL
    # single-rank DAG has no Pack
    assert sp.spmv_plan_validate(1, _codes(["start", "Pack", "yL", "end"]), smap, 1) == sp.SPMV_EPLAN
    assert sp.spmv_plan_validate(1, _codes(["start", "yL", "end"]), smap, 1) == sp.SPMV_EPLAN
    assert sp.spmv_plan_validate(1, _codes(["start", "yL", "end"]), None, 1) == sp.SPMV_OK


def test_explicit_unpack_on_other_stream_needs_stream_wait():
    """Table III, GPU -> GPU across streams: a record after Unpack and a
    stream wait before y_R."""
    smap = np.full(10, -1, np.int32)
    smap[[sp.SPMV_OP_PACK, sp.SPMV_OP_YL, sp.SPMV_OP_UNPACK, sp.SPMV_OP_YR]] = [0, 1, 0, 1]
    ops = _codes(BASE)
    i = ops.index(sp.SPMV_OP_YR)
    no_sync = ops[:i] + [sp.SPMV_OP_UNPACK] + ops[i:]
    assert sp.spmv_plan_validate(4, no_sync, smap, 2) == sp.SPMV_EPLAN
    with_sync = ops[:i] + [sp.SPMV_OP_UNPACK, sp.SPMV_CER_AFTER(sp.SPMV_OP_UNPACK),
                           sp.SPMV_CSWE_B4(sp.SPMV_OP_YR)] + ops[i:]
    assert sp.spmv_plan_validate(4, with_sync, smap, 2) == sp.SPMV_OK
    smap[sp.SPMV_OP_UNPACK] = 1    # same stream: the tokens become superfluous
    assert sp.spmv_plan_validate(4, with_sync, smap, 2) == sp.SPMV_EPLAN
    assert sp.spmv_plan_validate(4, no_sync, smap, 2) == sp.SPMV_OK


def test_stream_canonicalisation():
    A = gen.laplacian_3d7(8)
    smap = np.full(10, -1, np.int32)
    smap[[sp.SPMV_OP_PACK, sp.SPMV_OP_YL, sp.SPMV_OP_YR]] = [2, 0, 2]
    p = sp.spmv_plan_create(A, 2, 0, _codes(BASE), smap, 3, tune=HOST_ONLY)
    try:
        m = sp.spmv_plan_get_i32(p, sp.SPMV_I32_STREAM_MAP)
        # Pack is the first GPU op in BASE: stream 0; y_L next: stream 1
        assert (m[sp.SPMV_OP_PACK], m[sp.SPMV_OP_YL], m[sp.SPMV_OP_YR]) == (0, 1, 0)
        assert m[sp.SPMV_OP_UNPACK] == m[sp.SPMV_OP_YR]
    finally:
        sp.spmv_plan_destroy(p)


# ------------------------------------------------------------ share metadata

def _share_matches_oracle(A, P, r):
    ref = oracle.split(A, P, r)
    p = sp.spmv_plan_create(A, P, r, tune=HOST_ONLY)
    try:
        info = sp.spmv_plan_info(p)
        assert info["lo"] == ref["lo"] and info["n_loc"] == ref["n_loc"]
        g = lambda w: sp.spmv_plan_get_i32(p, w)
        pairs = [(sp.SPMV_I32_HALO_COLS, "H"), (sp.SPMV_I32_RECV_OFF, "recv_off"),
                 (sp.SPMV_I32_SEND_IDX, "send_idx"), (sp.SPMV_I32_SEND_OFF, "send_off"),
                 (sp.SPMV_I32_AL_PTR, "L_ptr"), (sp.SPMV_I32_AL_COLS, "L_col"),
                 (sp.SPMV_I32_AR_ROWS, "R_rows"), (sp.SPMV_I32_AR_PTR, "R_ptr"),
                 (sp.SPMV_I32_AR_COLS, "R_col")]
        for w, k in pairs:
            assert np.array_equal(g(w), ref[k]), k
        assert np.array_equal(g(sp.SPMV_I32_UNPACK_PERM), np.arange(ref["H"].size))
        for w, k in [(sp.SPMV_F64_AL_VAL, "L_val"), (sp.SPMV_F64_AR_VAL, "R_val")]:
            assert np.array_equal(sp.spmv_plan_get_f64(p, w).view(np.int64),
                                  ref[k].view(np.int64)), k
    finally:
        sp.spmv_plan_destroy(p)


@pytest.mark.parametrize("P", [1, 2, 3, 4, 7])
def test_share_metadata_banded(P):
    A = gen.banded_uniform(2000, 10, 500, seed=3)
    for r in range(P):
        _share_matches_oracle(A, P, r)


def test_share_metadata_stencils_and_powerlaw():
    _share_matches_oracle(gen.laplacian_3d7(16), 4, 1)
    _share_matches_oracle(gen.stencil_3d27(12, seed=3), 8, 3)
    _share_matches_oracle(gen.laplacian_2d5(64), 1, 0)
    A = gen.power_law(20000, seed=5)
    for r in (0, 5, 15):
        _share_matches_oracle(A, 16, r)


def test_share_metadata_more_ranks_than_rows():
    A = gen.laplacian_2d5(2, 2)      # 4 rows, 6 ranks: ranks 4, 5 own nothing
    for r in range(6):
        _share_matches_oracle(A, 6, r)


def test_malformed_csr_rejected():
    A = gen.laplacian_2d5(4)
    bad_cols = gen.CSR(A.n_rows, A.n_cols, A.row_ptr, A.col_idx.copy(), A.val)
    bad_cols.col_idx[3] = 99
    unsorted = gen.CSR(A.n_rows, A.n_cols, A.row_ptr, A.col_idx.copy(), A.val)
    unsorted.col_idx[[0, 1]] = unsorted.col_idx[[1, 0]]
    bad_ptr = gen.CSR(A.n_rows, A.n_cols, A.row_ptr.copy(), A.col_idx, A.val)
    bad_ptr.row_ptr[2] = bad_ptr.row_ptr[3] + 1
    for M in (bad_cols, unsorted, bad_ptr):
        with pytest.raises(sp.SpmvError) as e:
            sp.spmv_plan_create(M, 2, 0, tune=HOST_ONLY)
        assert e.value.code == sp.SPMV_ECSR
    with pytest.raises(sp.SpmvError) as e:
        sp.spmv_plan_create(A, 2, 2, tune=HOST_ONLY)
    assert e.value.code == sp.SPMV_EINVAL
    with pytest.raises(sp.SpmvError) as e:
        sp.spmv_plan_create(A, 2, 0, tune={"flags": sp.SPMV_F_HOST_ONLY, "lanes_local": 3})
    assert e.value.code == sp.SPMV_EINVAL


def test_host_only_plan_refuses_device_calls():
    A = gen.laplacian_3d7(8)
    p = sp.spmv_plan_create(A, 2, 1, tune=HOST_ONLY)
    try:
        for fn in (lambda: sp._lib.spmv_exec_resident(p, None, None, None),
                   lambda: sp._lib.spmv_exec_resident_part(p, 0, None, None, None),
                   lambda: sp._lib.spmv_plan_device_buffers(p, None, None, None, None)):
            assert fn() == sp.SPMV_ESTATE
    finally:
        sp.spmv_plan_destroy(p)


def test_resident_part_rejects_null_plan():
    assert sp._lib.spmv_exec_resident_part(None, 0, None, None, None) == sp.SPMV_EINVAL


def test_host_only_plan_refuses_exec():
    A = gen.laplacian_2d5(4)
    p = sp.spmv_plan_create(A, 1, 0, tune=HOST_ONLY)
    try:
        with pytest.raises(sp.SpmvError) as e:
            sp.spmv_exec(p, 0, 0)
        assert e.value.code == sp.SPMV_ESTATE
    finally:
        sp.spmv_plan_destroy(p)


def test_binding_rejects_bad_vectors_before_any_launch():
    """The binding checks x / y before calling the library: host arrays,
    CPU tensors, other dtypes, strided views, short tensors and missing
    vectors raise; nothing reaches a kernel (the plan is host-only, so a
    call that got through would return SPMV_ESTATE instead)."""
    import torch
    A = gen.laplacian_3d7(6)
    p = sp.spmv_plan_create(A, 2, 1, tune=HOST_ONLY)
    try:
        info = sp.spmv_plan_info(p)
        n = info["n_loc"]
        assert info["device"] == -1
        good_shape = torch.zeros(n, dtype=torch.float64)
        bad = [(np.zeros(n), TypeError),                                   # host numpy
               (good_shape, ValueError),                                   # CPU tensor
               (torch.zeros(n, dtype=torch.float32), ValueError),          # CPU, fp32
               ("not a tensor", TypeError),
               (None, ValueError)]                                         # missing
        for v, exc in bad:
            with pytest.raises(exc):
                sp.spmv_exec(p, v, 0)
            with pytest.raises(exc):
                sp.spmv_exec(p, 0, v)
            with pytest.raises(exc):
                sp.spmv_op_launch(p, sp.SPMV_OP_YL, v, 0)
            with pytest.raises(exc):
                sp.spmv_plan_time([p], [v], [0])
        # the remaining checks need the tensor to be on a GPU; their order
        # (device, dtype, contiguity, length) is exercised by the GPU tests
        with pytest.raises(ValueError):
            sp.spmv_plan_time([p], [0], [0, 0])
        # raw integer addresses pass the binding: the library then refuses the
        # host-only plan
        with pytest.raises(sp.SpmvError) as e:
            sp.spmv_exec(p, 1 << 20, 2 << 20)
        assert e.value.code == sp.SPMV_ESTATE
    finally:
        sp.spmv_plan_destroy(p)


def test_fused_unpack_is_the_default():
    A = gen.laplacian_3d7(8)
    for tune, fused in (({}, 1), ({"fuse_unpack": 1}, 1), ({"fuse_unpack": 2}, 0)):
        p = sp.spmv_plan_create(A, 4, 1, tune={"flags": sp.SPMV_F_HOST_ONLY, **tune})
        try:
            assert sp.spmv_plan_info(p)["fuse_unpack"] == fused
        finally:
            sp.spmv_plan_destroy(p)
    with pytest.raises(sp.SpmvError) as e:
        sp.spmv_plan_create(A, 4, 1, tune={"flags": sp.SPMV_F_HOST_ONLY, "fuse_unpack": 3})
    assert e.value.code == sp.SPMV_EINVAL


def test_default_plan_fuses_combine():
    A = gen.laplacian_3d7(8)
    p = sp.spmv_plan_create(A, 2, 1, tune=HOST_ONLY)
    try:
        info = sp.spmv_plan_info(p)
        assert info["fused_combine"] == 1
        # automatic kernel: stream CSR, window chunk 4 for 7-entry rows
        assert info["kernel_local"] == 2 and info["chunk_local"] == 4
    finally:
        sp.spmv_plan_destroy(p)
    p = sp.spmv_plan_create(A, 2, 1, tune={"flags": sp.SPMV_F_HOST_ONLY, "kernel_local": 1})
    try:
        info = sp.spmv_plan_info(p)
        assert info["kernel_local"] == 1 and info["lanes_local"] == 8
    finally:
        sp.spmv_plan_destroy(p)


def test_reorder_host_only():
    A = gen.laplacian_3d7(8)
    p = sp.spmv_plan_create(A, 2, 1, tune=HOST_ONLY)
    try:
        before = sp.spmv_plan_get_i32(p, sp.SPMV_I32_OP_ORDER).tolist()
        with pytest.raises(sp.SpmvError) as e:
            sp.spmv_plan_reorder(p, _codes(BASE[:-1]), None, 2)
        assert e.value.code == sp.SPMV_EPLAN
        assert sp.spmv_plan_get_i32(p, sp.SPMV_I32_OP_ORDER).tolist() == before
        ops, smap = sp.spmv_plan_space_get(2, 2, 17)
        sp.spmv_plan_reorder(p, ops, smap, 2)
        got = sp.spmv_plan_get_i32(p, sp.SPMV_I32_OP_ORDER).tolist()
        # the stored order has the implied Unpack inserted before y_R
        assert [t for t in got if t != sp.SPMV_OP_UNPACK] == ops.tolist()
        assert got.index(sp.SPMV_OP_UNPACK) == got.index(sp.SPMV_OP_YR) - 1
    finally:
        sp.spmv_plan_destroy(p)


def _check_tiles(rp, trow, tk, cap, maxr, vw):
    """Invariants the stream kernel relies on (its LDS indices stay inside
    the window and the row-pointer stage): tiles partition the rows in order,
    tile_k is the tile's first entry, a tile's entries fit the window from
    its first entry rounded down to vw unless it is a single row, and a tile
    has at most maxr rows."""
    n = rp.size - 1
    assert trow[0] == 0 and trow[-1] == n and np.all(np.diff(trow) >= 1) or n == 0
    assert np.array_equal(tk, rp[trow])
    for t in range(trow.size - 1):
        r0, r1 = trow[t], trow[t + 1]
        base = rp[r0] & ~(vw - 1)
        assert r1 - r0 <= maxr
        if r1 - r0 > 1:
            assert rp[r1] - base <= cap
        # maximal: the next row would not have fitted
        if r1 < n and r1 - r0 < maxr and rp[r0 + 1] - base <= cap:
            assert rp[r1 + 1] - base > cap


@pytest.mark.parametrize("chunk,width,lanes", [(4, 2, 1), (8, 2, 2), (8, 4, 4), (16, 4, 16),
                                               (16, 2, 8)])
def test_stream_tiles_invariants(chunk, width, lanes):
    for A, P, r in [(gen.power_law(30000, mean_len=40.0, seed=8), 4, 1),
                    (gen.power_law(20000, mean_len=300.0, seed=9), 2, 0),
                    (gen.laplacian_3d7(16), 4, 1), (gen.stencil_3d27(10, seed=3), 2, 1),
                    (gen.laplacian_2d5(2, 2), 6, 5)]:
        p = sp.spmv_plan_create(A, P, r, tune={"flags": sp.SPMV_F_HOST_ONLY, "kernel_local": 2,
                                               "kernel_remote": 2, "chunk_local": chunk,
                                               "chunk_remote": chunk, "width": width,
                                               "lanes_local": lanes, "lanes_remote": lanes,
                                               "form": 1})
        try:
            info = sp.spmv_plan_info(p)
            cap, maxr = 256 * chunk, 256 // lanes
            for rpw, trw, tkw in ((sp.SPMV_I32_AL_PTR, sp.SPMV_I32_TILE_ROW_L, sp.SPMV_I32_TILE_K_L),
                                  (sp.SPMV_I32_AR_PTR, sp.SPMV_I32_TILE_ROW_R, sp.SPMV_I32_TILE_K_R)):
                rp = sp.spmv_plan_get_i32(p, rpw).astype(np.int64)
                trow = sp.spmv_plan_get_i32(p, trw).astype(np.int64)
                tk = sp.spmv_plan_get_i32(p, tkw).astype(np.int64)
                _check_tiles(rp, trow, tk, cap, maxr, width)
            assert info["kernel_local"] == 2
        finally:
            sp.spmv_plan_destroy(p)


def test_batch_rejects_bad_plans_on_host():
    A = gen.laplacian_3d7(8)
    p = sp.spmv_plan_create(A, 2, 0, tune=HOST_ONLY)
    try:
        with pytest.raises(sp.SpmvError) as e:
            sp.spmv_batch_create([p])
        assert e.value.code == sp.SPMV_EINVAL
        with pytest.raises(sp.SpmvError) as e:
            sp.spmv_batch_create([])
        assert e.value.code == sp.SPMV_EINVAL
    finally:
        sp.spmv_plan_destroy(p)


def test_server_rejects_bad_options_on_host():
    for opts in ({"mode": 3}, {"chunk": 5}, {"budget_bytes": -1}):
        with pytest.raises(sp.SpmvError) as e:
            sp.spmv_server_create(opts)
        assert e.value.code == sp.SPMV_EINVAL


def _local_rows(A, P, r):
    lo = oracle.row_blocks(A.n_rows, P)
    a, b = int(lo[r]), int(lo[r + 1])
    rp = A.row_ptr[a:b + 1].astype(np.int64)
    return gen.CSR(b - a, A.n_cols, (rp - rp[0]).astype(np.int32),
                   A.col_idx[rp[0]:rp[-1]].copy(), A.val[rp[0]:rp[-1]].copy())


@pytest.mark.parametrize("P,r", [(4, 1), (16, 5), (3, 0), (6, 5)])
def test_local_plan_matches_global(P, r):
    """A plan built from the rank's own rows and the send lists equals the
    plan built from the global matrix (the send lists come from the oracle)."""
    A = gen.power_law(20000, seed=11) if P >= 6 else gen.banded_uniform(3000, 10, 750, seed=4)
    ref = oracle.split(A, P, r)
    pl = sp.spmv_plan_create_local(_local_rows(A, P, r), A.n_rows, P, r, ref["send_idx"],
                                   ref["send_off"], tune=HOST_ONLY)
    pg = sp.spmv_plan_create(A, P, r, tune=HOST_ONLY)
    try:
        for w in range(16):
            if w in (sp.SPMV_I32_OP_ORDER, sp.SPMV_I32_STREAM_MAP):
                continue
            assert np.array_equal(sp.spmv_plan_get_i32(pl, w), sp.spmv_plan_get_i32(pg, w)), w
        for w in (sp.SPMV_F64_AL_VAL, sp.SPMV_F64_AR_VAL):
            assert np.array_equal(sp.spmv_plan_get_f64(pl, w), sp.spmv_plan_get_f64(pg, w))
    finally:
        sp.spmv_plan_destroy(pl)
        sp.spmv_plan_destroy(pg)


def test_local_plan_rejects_bad_send_lists():
    A = gen.banded_uniform(3000, 10, 750, seed=4)
    P, r = 4, 1
    ref = oracle.split(A, P, r)
    loc = _local_rows(A, P, r)
    bad = []
    s = ref["send_idx"].copy()
    s[[0, 1]] = s[[1, 0]]                                   # not ascending
    bad.append((s, ref["send_off"]))
    s = ref["send_idx"].copy()
    s[-1] = 10 ** 6                                         # out of the rows
    bad.append((s, ref["send_off"]))
    off = ref["send_off"].copy()
    off[r + 1] += 1                                         # sends to itself
    bad.append((np.concatenate([ref["send_idx"], [0]]), np.maximum.accumulate(off)))
    for si, so in bad:
        with pytest.raises(sp.SpmvError) as e:
            sp.spmv_plan_create_local(loc, A.n_rows, P, r, si, so, tune=HOST_ONLY)
        assert e.value.code == sp.SPMV_EINVAL
    with pytest.raises(sp.SpmvError):      # wrong number of local rows
        sp.spmv_plan_create_local(_local_rows(A, 3, 0), A.n_rows, P, r, ref["send_idx"],
                                  ref["send_off"], tune=HOST_ONLY)


def test_power_law_share_structure():
    d = gen.power_law_share(200000, 16, 5, seed=3)
    loc = d["local"]
    loc.n_cols = d["n_global"]
    so = d["send_off"]
    assert so[0] == 0 and np.all(np.diff(so) >= 0) and so[6] == so[5]
    for q in range(16):
        seg = d["send_idx"][so[q]:so[q + 1]]
        assert np.all(np.diff(seg) > 0) and (seg.size == 0 or (seg.min() >= 0 and seg.max() < loc.n_rows))
    L = np.diff(loc.row_ptr)
    assert abs(L.mean() - 16) < 0.5
    # rank 0's ~12500*16 entries hit this 12500-column block with p = 1/16:
    # ~12500 uniform hits, of which 12500 * (1 - 1/e) distinct on average
    import math
    assert abs(np.diff(so)[0] - 12500 * (1 - math.exp(-1))) < 0.05 * 12500
    p = sp.spmv_plan_create_local(loc, d["n_global"], 16, 5, d["send_idx"], so, tune=HOST_ONLY)
    try:
        info = sp.spmv_plan_info(p)
        ref = oracle.split_local(loc, d["n_global"], 16, 5, d["send_idx"], so)
        assert info["n_halo"] == ref["H"].size and info["nnz_remote"] == ref["R_val"].size
    finally:
        sp.spmv_plan_destroy(p)


def test_column_slab_form_on_host():
    """Form 5: y_R in 8 column slabs, each a full set of packed tiles over
    every remote row (the concatenated tile arrays hold 8 runs from row 0 to
    the last remote row); y_L takes the automatic form; summing lanes at
    most 4; no remote rows or the vector kernel leave the packed or vector
    form."""
    def info(A, P, r, **tune):
        p = sp.spmv_plan_create(A, P, r, tune={"flags": sp.SPMV_F_HOST_ONLY, **tune})
        try:
            i = sp.spmv_plan_info(p)
            tr = tk = None
            if i["form_remote"] == 5:
                tr = sp.spmv_plan_get_i32(p, sp.SPMV_I32_TILE_ROW_R)
                tk = sp.spmv_plan_get_i32(p, sp.SPMV_I32_TILE_K_R)
            return i, tr, tk
        finally:
            sp.spmv_plan_destroy(p)
    A = gen.power_law(20000, seed=3)
    i0, _, _ = info(A, 4, 1)
    i, tr, tk = info(A, 4, 1, form=5)
    assert i0["form_remote"] == 1            # a halo far inside one XCD's L2
    assert i["form_remote"] == 5 and i["form_local"] == i0["form_local"]
    # about 2 entries per row per slab: one summing lane, tiles of 256 rows
    assert (i["lanes_remote"], i["rows_remote"]) == (1, 1)
    n_rr = i["n_remote_rows"]
    starts = np.flatnonzero(tr == 0)
    ends = np.flatnonzero(tr == n_rr)
    assert starts.size == 8 and ends.size == 8 and starts[0] == 0
    assert np.array_equal(starts[1:], ends[:-1] + 1) and ends[-1] == tr.size - 1
    assert tr.size == i["n_tiles_remote"] + 8
    total = 0
    for a, b in zip(starts, ends):
        assert np.all(np.diff(tr[a:b + 1]) > 0) and np.all(np.diff(tk[a:b + 1]) >= 0)
        assert tk[a] == 0
        total += int(tk[b])
    assert total == i["nnz_remote"]          # every remote entry in one slab
    assert np.diff(tr).max() <= 256
    # wide tiles (rows per thread > 1): up to rows * 256 rows, windows of
    # 256 * chunk entries (8 unless given), one summing lane; explicit rows
    # per thread with lanes > 1 are refused
    i4, tr4, tk4 = info(A, 4, 1, form=5, rows_remote=4)
    assert (i4["lanes_remote"], i4["rows_remote"], i4["chunk_remote"]) == (1, 4, 8)
    for a, b in zip(np.flatnonzero(tr4 == 0), np.flatnonzero(tr4 == n_rr)):
        rows, ents = np.diff(tr4[a:b + 1]), np.diff(tk4[a:b + 1])
        assert rows.max() <= 4 * 256 and np.all((ents <= 8 * 256) | (rows == 1))
    assert i4["n_tiles_remote"] < i["n_tiles_remote"]
    i8, _, _ = info(A, 4, 1, form=5, rows_remote=8, chunk_remote=16)
    assert (i8["rows_remote"], i8["chunk_remote"]) == (8, 16)
    with pytest.raises(sp.SpmvError):
        sp.spmv_plan_create(A, 4, 1, tune={"flags": sp.SPMV_F_HOST_ONLY, "form": 5,
                                           "lanes_remote": 2, "rows_remote": 2})
    # lanes beyond 4 are refused; no remote rows: packed; vector kernel: 0
    with pytest.raises(sp.SpmvError):
        sp.spmv_plan_create(A, 4, 1, tune={"flags": sp.SPMV_F_HOST_ONLY, "form": 5,
                                           "lanes_remote": 8})
    i2 = info(A, 4, 1, form=5, lanes_remote=2)[0]
    assert (i2["lanes_remote"], i2["rows_remote"]) == (2, 1)
    assert info(gen.laplacian_3d7(8), 1, 0, form=5)[0]["form_remote"] == 1
    assert info(A, 4, 1, form=5, kernel_remote=1)[0]["form_remote"] == 0
    with pytest.raises(sp.SpmvError):
        sp.spmv_plan_create(A, 4, 1, tune={"flags": sp.SPMV_F_HOST_ONLY, "form": 6})


def _wide_halo_share(n_half, seed=0):
    """Two ranks; each of rank 0's rows has one entry on its diagonal and
    one in rank 1's block, at distinct columns: rank 0's halo has n_half
    entries."""
    rng = np.random.default_rng(seed)
    n = 2 * n_half
    far = n_half + rng.permutation(n_half)
    ptr = [np.arange(0, 2 * n_half + 1, 2, dtype=np.int32),
           2 * n_half + np.arange(1, n_half + 1, dtype=np.int32)]
    col = np.empty(2 * n_half, np.int32)
    col[0::2] = np.arange(n_half)
    col[1::2] = far
    col = np.concatenate([col, np.arange(n_half, n, dtype=np.int32)])
    return gen.CSR(n, n, np.concatenate(ptr).astype(np.int32), col,
                   rng.standard_normal(col.size))


def test_column_slabs_automatic_beyond_one_l2():
    """The automatic form takes column slabs for y_R exactly when the halo
    (8 bytes per entry) is larger than one XCD's 4 MiB L2; an explicit
    form 1 keeps packed tiles; the vector kernel never slabs."""
    for n_half, slabs in ((524_288, False), (524_289, True)):
        A = _wide_halo_share(n_half)
        p = sp.spmv_plan_create(A, 2, 0, tune=HOST_ONLY)
        try:
            i = sp.spmv_plan_info(p)
            assert i["n_halo"] == n_half
            # one entry per row: below the limit the automatic sliced form
            assert i["form_remote"] == (5 if slabs else 2), n_half
            if slabs:   # one entry per row: one summing lane
                assert (i["lanes_remote"], i["rows_remote"]) == (1, 1)
        finally:
            sp.spmv_plan_destroy(p)
    A = _wide_halo_share(600_000)
    for tune, form in (({"form": 1}, 1), ({"form": 2}, 2), ({"kernel_remote": 1}, 0),
                       ({"form": 5}, 5)):
        p = sp.spmv_plan_create(A, 2, 0, tune={"flags": sp.SPMV_F_HOST_ONLY, **tune})
        try:
            assert sp.spmv_plan_info(p)["form_remote"] == form, tune
        finally:
            sp.spmv_plan_destroy(p)


def test_sliced_form_choice_on_host():
    """Automatic form: sliced ELL when every slice of 64 rows has one width
    of at most 8 (7-point share, its one-entry remote rows), with y_L's
    columns as 16-bit offsets from the row when they fit (form 3), packed
    tiles otherwise (27-point rows, uneven power-law rows), y_L's columns
    as 16-bit offsets from each tile's first row when they fit (form 4);
    explicit form 2 takes the sliced layout whenever padding stays within
    15%, form 3 moreover needs one width and offsets within 16 bits (else
    form 2), for y_L only; form 4 needs the tile offsets to fit (else 1)."""
    def info(A, P, r, **tune):
        p = sp.spmv_plan_create(A, P, r, tune={"flags": sp.SPMV_F_HOST_ONLY, **tune})
        try:
            return sp.spmv_plan_info(p)
        finally:
            sp.spmv_plan_destroy(p)
    i = info(gen.laplacian_3d7(32), 4, 1)
    assert (i["form_local"], i["form_remote"]) == (3, 2)
    assert i["n_slices_local"] == (i["n_loc"] + 63) // 64 and i["n_tiles_local"] == 0
    assert i["n_slices_remote"] == (i["n_remote_rows"] + 63) // 64
    assert i["chunk_local"] == 8 and i["chunk_remote"] == 4
    i = info(gen.laplacian_3d7(32), 4, 1, form=2)
    assert (i["form_local"], i["form_remote"]) == (2, 2) and i["chunk_local"] == 8
    i = info(gen.stencil_3d27(20, seed=3), 4, 1)
    assert i["form_local"] == 4 and i["n_slices_local"] == 0 and i["n_tiles_local"] > 0
    i = info(gen.stencil_3d27(20, seed=3), 4, 1, form=1)
    assert i["form_local"] == 1 and i["n_tiles_local"] > 0
    i = info(gen.laplacian_3d7(32), 4, 1, form=4)
    assert i["form_local"] == 4 and i["n_tiles_local"] > 0 and i["form_remote"] == 1
    i = info(gen.power_law(20000, seed=3), 4, 1, form=4)
    assert i["form_local"] == 4                      # 5,000 local columns: all fit
    i = info(gen.power_law(200000, seed=3), 2, 1, form=4)
    assert i["form_local"] == 1                      # columns far from the rows'
    i = info(gen.power_law(200000, seed=3), 2, 1)
    assert i["form_local"] == 1
    i = info(gen.stencil_3d27(20, seed=3), 4, 1, form=2)
    assert i["form_local"] == 2 and i["chunk_local"] == 16
    # slices of unequal widths (padding to one width > 15% on the small grid)
    i = info(gen.stencil_3d27(20, seed=3), 4, 1, form=3)
    assert i["form_local"] == 2
    i = info(gen.stencil_3d27(40, seed=3), 4, 1, form=3)
    assert i["form_local"] == 3 and i["chunk_local"] == 16 and i["form_remote"] == 2
    i = info(gen.stencil_3d27(40, seed=3), 4, 1, form=3, chunk_local=4)
    assert i["form_local"] == 3 and i["chunk_local"] == 8
    # offsets up to 40,000 do not fit 16 bits: the 32-bit sliced form stays
    i = info(gen.banded_uniform(90000, 4, 40000, seed=2), 1, 0, form=3)
    assert i["form_local"] == 2
    i = info(gen.banded_uniform(90000, 4, 30000, seed=2), 1, 0, form=3)
    assert i["form_local"] == 3
    i = info(gen.power_law(20000, seed=3), 4, 1, form=2)
    assert i["form_local"] == 1                      # padding far beyond 15%
    i = info(gen.power_law(20000, seed=3), 4, 1, form=3)
    assert i["form_local"] == 1
    i = info(gen.laplacian_3d7(32), 4, 1, form=1)
    assert i["form_local"] == 1 and i["n_tiles_local"] > 0
    i = info(gen.laplacian_3d7(32), 4, 1, kernel_local=1)
    assert i["form_local"] == 0
    # the 16-bit boundary: offsets of exactly +-32767 fit the sliced form,
    # +-32768 do not (-32768 marks padding); tiles add up to 255 rows
    def tri(d):
        return gen.three_diagonals(200000, d)
    assert info(tri(32767), 1, 0, form=3)["form_local"] == 3
    assert info(tri(32768), 1, 0, form=3)["form_local"] == 2
    assert info(tri(32767 - 255), 1, 0, form=4)["form_local"] == 4
    assert info(tri(32768), 1, 0, form=4)["form_local"] == 1
    # an empty local block (every entry remote): the 32-bit sliced form
    n = 256
    rows = np.arange(n)
    C = gen.CSR(n, n, np.arange(n + 1, dtype=np.int32), ((rows + n // 2) % n).astype(np.int32),
                np.ones(n))
    assert info(C, 2, 1)["form_local"] == 2
    assert info(C, 2, 1, form=3)["form_local"] == 2
    assert info(C, 2, 1, form=4)["form_local"] == 4
    with pytest.raises(sp.SpmvError):
        info(gen.laplacian_3d7(8), 4, 1, form=6)
