"""Monte-Carlo tree search (Sec. III-C): the oracle's search pinned against
what the paper fixes, then the library's search against the oracle.

Pins of the oracle (independent of the library):
* run to exhaustion it benchmarks every plan of the brute-force plan space
  exactly once (each rollout ends in a new plan);
* the exploitation value V stays in [0, 1] at every selection, and a fully
  explored child scores -inf and is never descended into again;
* selection stops at a node with a child that has no rollouts: the first
  rollouts create every child of the root's only child (start) before any
  of them is descended into;
* backpropagation: every node's rollout count and time range equal, by
  brute force over the rollout log, those of the plans below its prefix;
* the exploitation term steers the search to the subtree with the wide time
  range.

Parity: with the same random draws and candidate order the library's search
makes the same rollouts, in the same order, and ends with the same tree.
"""
import math
import zlib

import numpy as np
import pytest

import oracle
from oracle import search
import paper_2203_02530_amd as sp

from test_abi_host import CODE_OF, NAME_OF


def _draws(seed, n=200_000):
    return np.random.default_rng(seed).integers(0, 2**63, size=n, dtype=np.uint64)


def _abi_key(token, stream):
    return (CODE_OF[token], -1 if stream is None else stream)


def _index_of(S):
    """Library plan index of each oracle plan (by operation names)."""
    out = {}
    for i in range(sp.spmv_plan_space_count(4, S)):
        ops, smap = sp.spmv_plan_space_get(4, S, i)
        names = tuple(sp.spmv_op_name(int(o)) for o in ops)
        out[(names, (int(smap[sp.SPMV_OP_PACK]), int(smap[sp.SPMV_OP_YL]),
                     int(smap[sp.SPMV_OP_YR])))] = i
    return out


def _cost_table(S, seed):
    """Times with structure: plans that post the receive before Pack are
    slower, plus noise; distinct values so ranges are never degenerate."""
    idx = _index_of(S)
    rng = np.random.default_rng(seed)
    cost = np.empty(len(idx))
    for plan, i in idx.items():
        order = plan[0]
        cost[i] = 1.0 + 0.5 * (order.index("PostRecv") < order.index("Pack")) + rng.random()
    return idx, cost


# ------------------------------------------------------------ oracle pins

@pytest.mark.parametrize("S", [1, 2, 3])
def test_oracle_exhaustion_visits_every_plan_once(S):
    space = oracle.plan_space(S)
    log, root = search.mcts(lambda p: float(zlib.crc32(repr(p).encode()) % 997), S, 0,
                            _draws(S).tolist())
    plans = [p for p, _ in log]
    assert len(plans) == len(space) == oracle.plan_space_count_formula(S)
    assert set(plans) == space
    assert root.full and root.n == len(space)


def test_oracle_selection_values_and_full_subtrees():
    idx, cost = _cost_table(2, 3)
    seen = {"V": [], "full_scores": []}

    def trace(ev, data):
        if ev == "select":
            parent, child, V, score = data
            seen["V"].append(V)
            assert 0.0 <= V <= 1.0
            if child.full:
                assert score == -math.inf
                seen["full_scores"].append(score)
        else:
            # a rollout's path, reported before backpropagation: none of its
            # nodes was fully explored by the earlier rollouts
            assert not any(nd.full for nd in data), "descended into a fully explored subtree"

    log, root = search.mcts(lambda p: cost[idx[p]], 2, 0, _draws(5).tolist(), trace=trace)
    assert len(log) == len(idx)
    assert any(0.0 < v < 1.0 for v in seen["V"])       # the ratio branch is exercised
    assert seen["full_scores"]                          # -inf scores were met


def test_oracle_expands_every_child_before_descending():
    log, root = search.mcts(lambda p: 1.0, 2, 3, _draws(7).tolist())
    start = root.children[0]
    assert [ch.prefix[-1] for ch in start.children] and len(start.children) == 3
    second = {p[0][1] for p, _ in log}
    # the children of start are Pack (one stream so far), yL and PostRecv
    assert second == {"Pack", "yL", "PostRecv"}


def test_oracle_backprop_matches_brute_force():
    idx, cost = _cost_table(2, 11)
    log, root = search.mcts(lambda p: cost[idx[p]], 2, 300, _draws(13).tolist())
    for nd in search.walk(root):
        k = len(nd.prefix)
        below = [t for p, t in log if _prefix_of(p)[:k] == nd.prefix]
        assert nd.n == len(below)
        if below:
            assert nd.t_min == min(below) and nd.t_max == max(below)


def _prefix_of(plan):
    """The step tuple of a complete oracle plan (streams canonical)."""
    order, (s_pack, s_yl, s_yr) = plan
    streams = {"Pack": s_pack, "yL": s_yl, "yR": s_yr}
    return tuple((t, streams.get(t)) for t in order)


def test_oracle_exploitation_prefers_wide_subtree():
    """Times vary only among plans whose first operation after start is
    PostRecv; every other subtree has one constant time.  V then favours
    the PostRecv child once each child has two rollouts."""
    def cost(plan):
        order = plan[0]
        return 2.0 + (zlib.crc32(repr(plan).encode()) % 1000) / 1000.0 \
            if order[1] == "PostRecv" else 1.0
    share = sum(1 for p in oracle.plan_space(2) if p[0][1] == "PostRecv") / 2016
    log, _ = search.mcts(cost, 2, 300, _draws(17).tolist())
    frac = sum(1 for p, _ in log if p[0][1] == "PostRecv") / len(log)
    assert frac > share + 0.15, (frac, share)


# ------------------------------------------------------------ library parity

def _oracle_run(S, cost, idx, iterations, draws, c=math.sqrt(2.0)):
    log, root = search.mcts(lambda p: cost[idx[p]], S, iterations, draws.tolist(), c=c,
                            key=_abi_key)
    return [idx[p] for p, _ in log], [t for _, t in log], root


@pytest.mark.parametrize("S,iterations,seed", [(2, 0, 1), (2, 50, 2), (2, 400, 3),
                                               (3, 0, 4), (1, 0, 5)])
def test_library_search_matches_oracle(S, iterations, seed):
    idx, cost = _cost_table(S, seed)
    draws = _draws(100 + seed)
    r = sp.spmv_mcts_run_table(4, cost, iterations=iterations, n_streams=S, rand=draws)
    ref_idx, ref_t, root = _oracle_run(S, cost, idx, iterations, draws)
    assert r["index"].tolist() == ref_idx
    assert r["time"].tolist() == ref_t
    # the same tree: node statistics per prefix
    nodes = r["nodes"]
    lib = {}
    prefix = {0: ()}
    for i in range(1, len(nodes)):
        nd = nodes[i]
        st = None if nd["stream"] < 0 else int(nd["stream"])
        prefix[i] = prefix[int(nd["parent"])] + ((NAME_OF.get(int(nd["token"])) or
                                                   sp.spmv_op_name(int(nd["token"])), st),)
        lib[prefix[i]] = (int(nd["n"]), float(nd["t_min"]), float(nd["t_max"]), int(nd["full"]))
    ref = {nd.prefix: (nd.n, nd.t_min, nd.t_max, int(nd.full))
           for nd in search.walk(root) if nd.prefix}
    assert lib == ref
    assert (int(nodes[0]["n"]), int(nodes[0]["full"])) == (root.n, int(root.full))


def test_library_search_other_exploration_constant():
    idx, cost = _cost_table(2, 21)
    draws = _draws(21)
    r = sp.spmv_mcts_run_table(4, cost, iterations=200, c=0.25, rand=draws)
    ref_idx, _, _ = _oracle_run(2, cost, idx, 200, draws, c=0.25)
    assert r["index"].tolist() == ref_idx


def test_library_search_seeded_generator_exhausts():
    cost = np.linspace(1.0, 2.0, 2016)
    r = sp.spmv_mcts_run_table(4, cost, seed=99)
    assert sorted(r["index"].tolist()) == list(range(2016))
    again = sp.spmv_mcts_run_table(4, cost, seed=99)
    assert again["index"].tolist() == r["index"].tolist()      # deterministic


def test_library_search_single_rank():
    r = sp.spmv_mcts_run_table(1, np.array([3.0]))
    assert r["index"].tolist() == [0] and r["time"].tolist() == [3.0]


def test_library_search_errors():
    cost = np.ones(2016)
    with pytest.raises(sp.SpmvError):
        sp.spmv_mcts_run_table(4, np.ones(5))                  # wrong table size
    with pytest.raises(sp.SpmvError):
        sp.spmv_mcts_run_table(4, cost, rand=np.array([1, 2, 3], np.uint64))   # draws run out
    with pytest.raises(sp.SpmvError):
        sp.spmv_mcts_run_table(4, cost, iterations=-1)
    with pytest.raises(sp.SpmvError):
        sp.spmv_mcts_run_table(4, cost, n_streams=99)


def test_device_search_on_host_only_plans_is_an_error():
    """The device search needs executable plans: host-only plans give
    SPMV_ESTATE from the first rollout's timing (and nothing is corrupted on
    the way: the prefix undo of a synchronisation token touches no stream)."""
    import gen
    A = gen.banded_uniform(2000, 7, 300, seed=4)
    plans = [sp.spmv_plan_create(A, 4, 1, None, None, 2, {"flags": sp.SPMV_F_HOST_ONLY})
             for _ in range(2)]
    try:
        # raw addresses pass the binding's checks (host arrays would not);
        # the library refuses the host-only plans before any launch
        xs = [1 << 20 for _ in plans]
        ys = [2 << 20 for _ in plans]
        with pytest.raises(sp.SpmvError) as e:
            sp.spmv_mcts_run(plans, xs, ys, None, iterations=5, seed=5, t_measure=0.001)
        assert e.value.code == sp.SPMV_ESTATE
        # the enumeration itself is unchanged
        assert sp.spmv_plan_space_count(4, 3) == 504 * 5
    finally:
        for p in plans:
            sp.spmv_plan_destroy(p)
