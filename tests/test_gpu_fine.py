"""Fine-grained programs on the device: per-peer Pack, copies and waits give
the bits of the coarse program (halo buffers bit-exact, y identical and
within tolerance of the oracle) for the default order and for orders drawn
by the tree search, and the device-timed search over the fine DAG."""
import numpy as np
import pytest

import gen
import oracle
import paper_2203_02530_amd as sp

from gpu_util import assert_share_parity, bits, log, run_share

pytestmark = pytest.mark.gpu

CASES = [("laplace3d_48_p4r1", lambda: gen.laplacian_3d7(48), 4, 1, 3),
         ("banded_60k_p4r2", lambda: gen.banded_uniform(60000, 10, 15000, seed=8), 4, 2, 9),
         ("powerlaw_40k_p6r3", lambda: gen.power_law(40000, seed=21), 6, 3, 22),
         ("stencil27_30_p8r3", lambda: gen.stencil_3d27(30, seed=5), 8, 3, 6)]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_fine_orders_match_coarse(case):
    name, build, P, r, seed = CASES[case]
    log(f"fine orders {name}")
    A = build()
    x = gen.x_normal(A.n_cols, seed)
    ref = oracle.share_reference(A, P, r, x)
    coarse, _ = run_share(A, P, r, x, ref=ref)
    assert_share_parity(coarse, ref)
    plan = sp.spmv_plan_create(A, P, r, None, None, 2)
    try:
        sp.spmv_plan_set_fine(plan)                       # default fine order
        res, _ = run_share(A, P, r, x, ref=ref, plan=plan)
        assert res["info"]["fine"] == 1
        assert_share_parity(res, ref)
        assert np.array_equal(bits(res["y"]), bits(coarse["y"]))
        # orders and stream maps drawn by the search (random costs)
        rng = np.random.default_rng(seed)
        draws = sp.spmv_mcts_run_seq(plan, fine=True, iterations=12, seed=seed,
                                     cost=lambda a, b: float(rng.random()))
        for ops, sts in zip(draws["ops"], draws["streams"]):
            sp.spmv_plan_set_fine(plan, ops, sts)
            res, _ = run_share(A, P, r, x, ref=ref, plan=plan)
            assert np.array_equal(bits(res["outbox"]), bits(ref["sendbuf"]))
            assert np.array_equal(bits(res["x_halo"]), bits(ref["inbox"]))
            assert np.array_equal(bits(res["y"]), bits(coarse["y"]))
        # and back to a coarse order
        ops, smap = sp.spmv_plan_space_get(P, 2, 100)
        sp.spmv_plan_reorder(plan, ops, smap, 2)
        res, _ = run_share(A, P, r, x, ref=ref, plan=plan)
        assert res["info"]["fine"] == 0
        assert np.array_equal(bits(res["y"]), bits(coarse["y"]))
    finally:
        sp.spmv_plan_destroy(plan)


def test_fine_device_search():
    import torch
    A = gen.laplacian_3d7(48)
    x = gen.x_normal(A.n_cols, 5)
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
        log("fine device search: 30 rollouts")
        res = sp.spmv_mcts_run_seq(plans, xs, ys, torch.cuda.current_stream(), fine=True,
                                   iterations=30, seed=3, t_measure=0.002)
        seqs = {(tuple(o), tuple(s)) for o, s in zip(res["ops"].tolist(), res["streams"].tolist())}
        assert len(seqs) == 30
        assert np.all(res["time"] > 0) and np.all(res["time"] < 0.002)
        assert res["nodes"][0]["n"] == 30
        # plans are left in the last rollout's order and still compute y
        last = res["ops"][-1]
        for p in plans:
            assert sp.spmv_plan_info(p)["fine"] == 1
            assert sp.spmv_plan_get_i32(p, sp.SPMV_I32_OP_ORDER).tolist() == last.tolist()
            out, _ = run_share(A, P, r, x, ref=ref, plan=p)
            assert_share_parity(out, ref)
    finally:
        for p in plans:
            sp.spmv_plan_destroy(p)
