"""The tree search timing rollouts on the device (Sec. III-C with the
benchmark protocol of Sec. III-C3): every rollout is a distinct plan of the
space, its time comes from real executions, and the plans still compute the
oracle's y afterwards."""
import numpy as np
import pytest

import gen
import oracle
import paper_2203_02530_amd as sp

from gpu_util import assert_share_parity, bits, log, run_share

pytestmark = pytest.mark.gpu


def test_device_search_rollouts():
    import torch
    A = gen.banded_uniform(20000, 10, 5000, seed=31)
    x = gen.x_normal(A.n_cols, 32)
    P, r = 4, 1
    ref = oracle.share_reference(A, P, r, x)
    plans = [sp.spmv_plan_create(A, P, r, None, None, 2) for _ in range(2)]
    try:
        xs, ys = [], []
        for p in plans:
            info = sp.spmv_plan_info(p)
            lo, n = info["lo"], info["n_loc"]
            sp.spmv_plan_inbox(p)[:] = ref["inbox"]
            xs.append(torch.from_numpy(x[lo:lo + n].copy()).cuda())
            ys.append(torch.empty(n, dtype=torch.float64, device="cuda"))
        torch.cuda.synchronize()
        log("device search: 40 rollouts")
        res = sp.spmv_mcts_run(plans, xs, ys, torch.cuda.current_stream(), iterations=40,
                               seed=5, t_measure=0.002)
        idx, t = res["index"], res["time"]
        assert idx.size == 40 and len(set(idx.tolist())) == 40
        assert np.all((idx >= 0) & (idx < 2016))
        assert np.all(t > 0) and np.all(t < 0.002)
        nodes = res["nodes"]
        assert nodes[0]["n"] == 40
        assert nodes[0]["t_min"] == t.min() and nodes[0]["t_max"] == t.max()
        # the plans are left in the last rollout's order and still compute y
        first = None
        for p in plans:
            out, _ = run_share(A, P, r, x, ref=ref, plan=p)
            assert_share_parity(out, ref)
            if first is None:
                first = bits(out["y"])
            assert np.array_equal(bits(out["y"]), first)
        ops, smap = sp.spmv_plan_space_get(P, 2, int(idx[-1]))
        sp.spmv_plan_validate(P, ops, smap, 2)
        got = sp.spmv_plan_get_i32(plans[0], sp.SPMV_I32_STREAM_MAP)
        for v in (sp.SPMV_OP_PACK, sp.SPMV_OP_YL, sp.SPMV_OP_YR):
            assert got[v] == smap[v]
    finally:
        for p in plans:
            sp.spmv_plan_destroy(p)


def test_device_search_matches_table_replay():
    """Replaying the device search's own times as a cost table reproduces
    its rollouts (same draws): the search depends on the times only."""
    import torch
    A = gen.laplacian_2d5(48)
    x = gen.x_normal(A.n_cols, 3)
    P, r = 4, 2
    ref = oracle.share_reference(A, P, r, x)
    plan = sp.spmv_plan_create(A, P, r, None, None, 2)
    try:
        info = sp.spmv_plan_info(plan)
        lo, n = info["lo"], info["n_loc"]
        sp.spmv_plan_inbox(plan)[:] = ref["inbox"]
        xd = torch.from_numpy(x[lo:lo + n].copy()).cuda()
        yd = torch.empty(n, dtype=torch.float64, device="cuda")
        draws = np.random.default_rng(8).integers(0, 2**63, size=4000, dtype=np.uint64)
        torch.cuda.synchronize()
        res = sp.spmv_mcts_run(plan, xd, yd, torch.cuda.current_stream(), iterations=60,
                               t_measure=0.001, rand=draws)
        cost = np.full(2016, np.inf)
        cost[res["index"]] = res["time"]
        rep = sp.spmv_mcts_run_table(P, cost, iterations=60, rand=draws)
        assert rep["index"].tolist() == res["index"].tolist()
    finally:
        sp.spmv_plan_destroy(plan)
