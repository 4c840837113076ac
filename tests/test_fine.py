"""The fine-grained program (Sec. III-A: one Pack / PostSend / WaitSend per
destination, one PostRecv / WaitRecv per source) on the host: its DAG and
program count against the oracle's, its single-peer case against the
coarse plan space, order validation, and the tree search over it against
the oracle's search."""
import zlib

import numpy as np
import pytest

import gen
import oracle
from oracle import fine as ofine
from oracle import search
import paper_2203_02530_amd as sp

HOST = {"flags": sp.SPMV_F_HOST_ONLY}


def _plan(A, P, r):
    return sp.spmv_plan_create(A, P, r, tune=HOST)


def _names(codes):
    return [sp.spmv_op_name(int(c)) for c in codes]


SHARES = [(gen.laplacian_3d7(12), 4, 1),          # two neighbours
          (gen.laplacian_3d7(12), 2, 0),          # one neighbour
          (gen.banded_uniform(3000, 6, 900, seed=3), 4, 2),
          (gen.power_law(600, mean_len=3.0, seed=5), 3, 1)]


@pytest.mark.parametrize("case", range(len(SHARES)))
def test_fine_dag_and_count_match_oracle(case):
    A, P, r = SHARES[case]
    split = oracle.split(A, P, r)
    dag = ofine.fine_dag(split, r)
    p = _plan(A, P, r)
    try:
        assert sorted(_names(sp.spmv_fine_tokens(p))) == sorted(dag.tokens)
        for S in (1, 2, 3):
            assert sp.spmv_fine_count(p, S) == ofine.count_programs(dag, S)
    finally:
        sp.spmv_plan_destroy(p)


def test_two_neighbour_count_closed_form():
    """Two destinations and two sources (the 7-point interior share): the
    orders interleave the chains Pack..WaitSend (5 tokens) twice, PostRecv,
    WaitRecv twice, yL, and yR after both WaitRecv; 4 GPU vertices give 8
    canonical stream maps on two streams."""
    A, P, r = SHARES[0]
    p = _plan(A, P, r)
    try:
        from math import factorial as f
        # 16 tokens between start and end: two send chains of 5, the receive
        # part (two chains of 2 then yR: 4!/(2!2!) = 6 orders) and yL
        closed = f(16) // (f(5) * f(5) * f(5) * f(1)) * 6
        orders = ofine.count_orders(ofine.fine_dag(oracle.split(A, P, r), r))
        assert orders == closed == 72_648_576
        assert sp.spmv_fine_count(p, 2) == orders * 8 == 581_188_608
    finally:
        sp.spmv_plan_destroy(p)


def test_single_peer_fine_space_is_the_coarse_space():
    A, P, r = SHARES[1]
    p = _plan(A, P, r)
    try:
        assert sp.spmv_fine_count(p, 2) == sp.spmv_plan_space_count(P, 2) == 2016
        res = sp.spmv_mcts_run_seq(p, fine=True, cost=lambda a, b: 1.0, seed=4)
        plans = set()
        for ops, sts in zip(res["ops"], res["streams"]):
            names = tuple(n.split("[")[0] for n in _names(ops))
            st = {n: int(s) for n, s in zip(names, sts) if s >= 0}
            plans.add((names, (st["Pack"], st["yL"], st["yR"])))
        assert len(plans) == 2016 and plans == oracle.plan_space(2)
    finally:
        sp.spmv_plan_destroy(p)


def test_fine_validation():
    A, P, r = SHARES[0]
    p = _plan(A, P, r)
    try:
        ops, sts = sp.spmv_fine_default(p)
        assert sp.spmv_fine_validate(p, ops, sts) == sp.SPMV_OK
        names = _names(ops)
        assert names[0] == "start" and names[-1] == "end"
        # every dependence of the oracle's DAG is respected by the default
        dag = ofine.fine_dag(oracle.split(A, P, r), r)
        pos = {n: i for i, n in enumerate(names)}
        assert all(pos[u] < pos[t] for t in names for u in dag.need[t])

        def bad(o, s=sts, code=sp.SPMV_EPLAN):
            with pytest.raises(sp.SpmvError) as e:
                sp.spmv_fine_validate(p, o, s)
            assert e.value.code == code
        i_cer, i_ces = names.index("CER-after-Pack[0]"), names.index("CES-b4-PostSend[0]")
        o = ops.copy()
        o[i_cer], o[i_ces] = o[i_ces], o[i_cer]                 # wait before its record
        bad(o)
        i_ps = names.index("PostSend[2]")
        o = np.delete(ops, i_ps)                                 # a token missing
        bad(o, np.delete(sts, i_ps))
        o = ops.copy()
        o[names.index("WaitSend[0]")] = ops[names.index("WaitSend[2]")]   # a token twice
        bad(o)
        i_yr = names.index("yR")
        o = list(ops)
        o.insert(names.index("WaitRecv[0]"), o.pop(i_yr))        # yR before WaitRecv[0]
        s2 = list(sts)
        s2.insert(names.index("WaitRecv[0]"), s2.pop(i_yr))
        bad(np.array(o), np.array(s2))
        s3 = sts.copy()
        s3[names.index("Pack[0]")] = 5                           # stream out of range
        bad(ops, s3)
        bad(np.array([0, 9]), np.array([-1, -1]))
        # the order can be made the plan's, and the coarse one restored
        sp.spmv_plan_set_fine(p, ops, sts)
        assert sp.spmv_plan_info(p)["fine"] == 1
        assert _names(sp.spmv_plan_get_i32(p, sp.SPMV_I32_OP_ORDER)) == names
        st = sp.spmv_plan_get_i32(p, sp.SPMV_I32_OP_STREAM)
        assert [int(x) for x in st] == [int(x) for x in sts]     # already canonical
        c_ops, c_map = sp.spmv_plan_space_get(P, 2, 0)
        sp.spmv_plan_reorder(p, c_ops, c_map, 2)
        assert sp.spmv_plan_info(p)["fine"] == 0
    finally:
        sp.spmv_plan_destroy(p)


def test_single_rank_has_no_fine_dag():
    A = gen.laplacian_2d5(16)
    p = _plan(A, 1, 0)
    try:
        with pytest.raises(sp.SpmvError):
            sp.spmv_fine_tokens(p)
        with pytest.raises(sp.SpmvError):
            sp.spmv_plan_set_fine(p)
    finally:
        sp.spmv_plan_destroy(p)


def _crc_cost(names, streams):
    key = "|".join(f"{n}:{s}" for n, s in zip(names, streams))
    return float(zlib.crc32(key.encode()) % 1000) / 1000.0 + 1.0


@pytest.mark.parametrize("case,iterations", [(0, 300), (3, 200), (1, 0)])
def test_fine_search_matches_oracle(case, iterations):
    A, P, r = SHARES[case]
    dag = ofine.fine_dag(oracle.split(A, P, r), r)
    p = _plan(A, P, r)
    try:
        code = {sp.spmv_op_name(int(c)): int(c) for c in sp.spmv_fine_tokens(p)}
        draws = np.random.default_rng(case + 10).integers(0, 2**63, size=200_000, dtype=np.uint64)
        res = sp.spmv_mcts_run_seq(
            p, fine=True, iterations=iterations, rand=draws,
            cost=lambda a, b: _crc_cost(_names(a), [int(x) for x in b]))
        log, root = search.mcts(
            lambda pre: _crc_cost([t for t, _ in pre], [-1 if s is None else s for _, s in pre]),
            2, iterations, draws.tolist(), dag=dag,
            key=lambda t, s: (code[t], -1 if s is None else s))
        assert len(log) == len(res["time"])
        for (pre, t), ops, sts, tt in zip(log, res["ops"], res["streams"], res["time"]):
            assert _names(ops) == [n for n, _ in pre]
            assert [int(x) for x in sts] == [-1 if s is None else s for _, s in pre]
            assert tt == t
        if iterations == 0:
            assert len(log) == ofine.count_programs(dag, 2)
    finally:
        sp.spmv_plan_destroy(p)


def test_coarse_sequence_search_matches_index_search():
    """The sequence form of the search over the coarse DAG makes the same
    rollouts as the plan-index form."""
    A, P, r = SHARES[0]
    p = _plan(A, P, r)
    try:
        n = sp.spmv_plan_space_count(P, 2)
        cost = np.random.default_rng(1).random(n)
        index = {}
        for i in range(n):
            ops, smap = sp.spmv_plan_space_get(P, 2, i)
            st = tuple(int(smap[o]) if o in (sp.SPMV_OP_PACK, sp.SPMV_OP_YL, sp.SPMV_OP_YR)
                       else -1 for o in ops)
            index[(tuple(int(o) for o in ops), st)] = i
        draws = np.random.default_rng(2).integers(0, 2**63, size=50_000, dtype=np.uint64)
        a = sp.spmv_mcts_run_table(P, cost, iterations=150, rand=draws)
        b = sp.spmv_mcts_run_seq(p, fine=False, iterations=150, rand=draws,
                                 cost=lambda o, s: cost[index[(tuple(int(x) for x in o),
                                                               tuple(int(x) for x in s))]])
        got = [index[(tuple(int(x) for x in o), tuple(int(x) for x in s))]
               for o, s in zip(b["ops"], b["streams"])]
        assert got == a["index"].tolist()
    finally:
        sp.spmv_plan_destroy(p)
