"""spmv_exec_static: the exec whose intermediate data lives in the library's
fixed per-device scratch array.  Its results must equal spmv_exec's bit for
bit (same kernels, same order), on consecutive calls over plans of
different sizes, and meet the oracle's bar; a plan needing more scratch
than the array holds is refused before anything runs."""
import numpy as np
import pytest

import gen
import oracle
import paper_2203_02530_amd as sp
from gpu_util import assert_share_parity, bits, log


def _wide_halo_share(n_half, seed=0):
    """Two ranks; each of rank 0's rows has its diagonal entry and one entry
    at a distinct column of rank 1's block: rank 0's halo has n_half entries
    and every row is a remote row."""
    rng = np.random.default_rng(seed)
    n = 2 * n_half
    ptr = np.concatenate([np.arange(0, 2 * n_half + 1, 2),
                          2 * n_half + np.arange(1, n_half + 1)]).astype(np.int32)
    col = np.empty(2 * n_half, np.int32)
    col[0::2] = np.arange(n_half)
    col[1::2] = n_half + rng.permutation(n_half)
    col = np.concatenate([col, np.arange(n_half, n, dtype=np.int32)])
    return gen.CSR(n, n, ptr, col, rng.standard_normal(col.size))


def test_static_scratch_size_limit_on_host():
    """The size check runs first (host-only plans reach it without a GPU):
    4,000,000 halo entries and remote rows (64 MB of receive buffer and
    partial sums) fit the 64 MiB array, 4,300,000 do not."""
    assert sp.spmv_static_scratch_bytes() == 64 << 20
    for n_half, fits in ((4_000_000, True), (4_300_000, False)):
        A = _wide_halo_share(n_half)
        p = sp.spmv_plan_create(A, 2, 0, tune={"flags": sp.SPMV_F_HOST_ONLY, "form": 1})
        try:
            info = sp.spmv_plan_info(p)
            assert info["n_halo"] == n_half and info["n_remote_rows"] == n_half
            assert info["fuse_unpack"] == 1
            rc = sp._lib.spmv_exec_static(p, None, None, None)
            msg = sp._lib.spmv_last_error().decode()
            if fits:
                assert rc == sp.SPMV_ESTATE, msg
            else:
                assert rc == sp.SPMV_EINVAL and "scratch" in msg, msg
        finally:
            sp.spmv_plan_destroy(p)


def _run(plan, x, exec_fn):
    import torch
    info = sp.spmv_plan_info(plan)
    lo, n = info["lo"], info["n_loc"]
    xd = torch.from_numpy(np.ascontiguousarray(x[lo:lo + n])).cuda()
    yd = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    exec_fn(plan, xd, yd, torch.cuda.current_stream())
    return yd.cpu().numpy(), sp.spmv_plan_outbox(plan).copy()


@pytest.mark.gpu
def test_static_exec_equals_exec():
    """Two calls in a row, the second on a smaller share: the column-slab
    power-law share (slab partial sums and a combine step in scratch), then
    a 7-point share (fused combine); each equals spmv_exec bit for bit and
    meets the oracle's bar.  A regular exec after the static ones still
    uses the plan's own buffers."""
    import torch
    assert torch.cuda.is_available()
    cases = [(gen.power_law(60000, seed=21), 4, 2, 31, {"form": 5, "fuse_unpack": 2}),
             (gen.laplacian_3d7(16), 4, 1, 2, {})]
    for A, P, r, seed, tune in cases:
        x = gen.x_normal(A.n_cols, seed)
        ref = oracle.share_reference(A, P, r, x)
        for idx in (7, 2003):   # a combine step at end, then y_R adding into y
            ops, smap = sp.spmv_plan_space_get(P, 2, idx)
            plan = sp.spmv_plan_create(A, P, r, ops, smap, 2, tune)
            try:
                info = sp.spmv_plan_info(plan)
                log(f"static exec n={A.n_rows} P={P} r={r} plan {idx} "
                    f"form_remote={info['form_remote']} fused_combine={info['fused_combine']}")
                sp.spmv_plan_inbox(plan)[:] = ref["inbox"]
                y_st, out_st = _run(plan, x, sp.spmv_exec_static)
                y_ex, out_ex = _run(plan, x, sp.spmv_exec)
                assert np.array_equal(bits(y_st), bits(y_ex))
                assert np.array_equal(bits(out_st), bits(ref["sendbuf"]))
                assert np.array_equal(bits(out_ex), bits(ref["sendbuf"]))
                res = dict(info=info, y=y_st, outbox=out_st,
                           recvbuf=sp.spmv_plan_get_f64(plan, sp.SPMV_F64_RECVBUF),
                           x_halo=sp.spmv_plan_get_f64(plan, sp.SPMV_F64_X_HALO),
                           sendbuf=sp.spmv_plan_get_f64(plan, sp.SPMV_F64_SENDBUF))
                assert_share_parity(res, ref)
            finally:
                sp.spmv_plan_destroy(plan)
