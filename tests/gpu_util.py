"""Helpers of the GPU parity tests: run one rank share through the C ABI."""
import sys

import numpy as np

import oracle
import paper_2203_02530_amd as sp


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def run_share(A, P, r, x, op_order=None, stream_map=None, n_streams=2, tune=None, ref=None,
              plan=None, keep_plan=False):
    """Execute rank r's share with the library; the inbox is filled from the
    oracle's halo values.  Returns (result dict, oracle reference dict)."""
    import torch
    ref = oracle.share_reference(A, P, r, x) if ref is None else ref
    own = plan is None
    if own:
        plan = sp.spmv_plan_create(A, P, r, op_order, stream_map, n_streams, tune)
    try:
        info = sp.spmv_plan_info(plan)
        lo, n = info["lo"], info["n_loc"]
        inbox = sp.spmv_plan_inbox(plan)
        inbox[:] = ref["inbox"]
        xd = torch.from_numpy(np.ascontiguousarray(x[lo:lo + n])).cuda()
        yd = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        sp.spmv_exec(plan, xd if n else None, yd if n else None, torch.cuda.current_stream())
        out = dict(info=info, y=yd.cpu().numpy(),
                   outbox=sp.spmv_plan_outbox(plan).copy(),
                   recvbuf=sp.spmv_plan_get_f64(plan, sp.SPMV_F64_RECVBUF),
                   x_halo=sp.spmv_plan_get_f64(plan, sp.SPMV_F64_X_HALO),
                   sendbuf=sp.spmv_plan_get_f64(plan, sp.SPMV_F64_SENDBUF))
        if keep_plan:
            out["plan"] = plan
        return out, ref
    finally:
        if own and not keep_plan:
            sp.spmv_plan_destroy(plan)


def bits(a):
    return np.ascontiguousarray(a, np.float64).view(np.int64)


def assert_share_parity(res, ref, rel=1e-12):
    """Halo contents bit-exact, y within rel*(|A||x|)_i per row."""
    assert np.array_equal(bits(res["outbox"]), bits(ref["sendbuf"]))
    assert np.array_equal(bits(res["sendbuf"]), bits(ref["sendbuf"]))
    assert np.array_equal(bits(res["recvbuf"]), bits(ref["inbox"]))
    assert np.array_equal(bits(res["x_halo"]), bits(ref["inbox"]))
    ok = oracle.within_tolerance(res["y"], ref["y"], ref["absax"], rel)
    bad = np.flatnonzero(~ok)
    assert bad.size == 0, (bad[:10], res["y"][bad[:10]], ref["y"][bad[:10]])
