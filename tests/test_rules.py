"""Design-rule generation (Sec. IV): class labels, pairwise features, CART
with Alg. 1, rule sets, and the Table V accuracy experiment.

The oracle's labelling (plain loops) is pinned by hand-computed
convolutions, peaks and prominences and by staircases whose classes are
known; the library's labelling (numpy + scipy) must then give the same
labels, bit for bit, on integer-valued times (every sum exact on both sides).
Features are pinned by a closed-form count of the varying pairs over the
full space.
"""
import numpy as np
import pytest

from oracle import rules as orules
import paper_2203_02530_amd as sp
from paper_2203_02530_amd import rules


# ------------------------------------------------------------ oracle pins

def test_oracle_step_conv_by_hand():
    c, first = orules.step_conv([0, 0, 1, 1], 1)
    assert (c, first) == ([0.0, 1.0, 0.0], 0)
    c, first = orules.step_conv([0, 0, 0, 5, 5, 5], 2)
    assert (c, first) == ([5.0, 10.0, 5.0], 1)
    assert orules.step_conv([1, 2, 3], 2) == ([], 1)


def test_oracle_peaks_by_hand():
    assert orules.local_peaks([0, 3, 1, 4, 0]) == [1, 3]
    assert orules.local_peaks([0, 2, 2, 2, 0]) == [2]          # flat top: middle
    assert orules.local_peaks([0, 2, 2, 2, 2, 0]) == [2]       # rounded down
    assert orules.local_peaks([0, 2, 2, 3, 0]) == [3]
    assert orules.local_peaks([0, 1, 1]) == []                 # no fall after the top
    assert orules.local_peaks([0, 1, 2]) == []
    assert orules.local_peaks([3, 1, 0]) == []                 # ends are never peaks


def test_oracle_prominence_by_hand():
    assert orules.prominence([0, 3, 1, 4, 0], 1) == 2
    assert orules.prominence([0, 3, 1, 4, 0], 3) == 4
    x = [2, 7, 3, 5, 1, 6, 0]
    assert [orules.prominence(x, p) for p in orules.local_peaks(x)] == [5, 2, 5]


def test_oracle_staircase_equal_jumps_gives_every_class():
    t = [10.0] * 700 + [20.0] * 800 + [30.0] * 516
    perm = np.random.default_rng(0).permutation(len(t))
    shuffled = [t[i] for i in perm]
    lab, bounds = orules.labels(shuffled)
    assert bounds == [700, 1500]
    assert lab == [int(v // 10) - 1 for v in shuffled]


def test_oracle_staircase_keeps_only_top_percentile():
    """Two unequal jumps: the 98th percentile of two prominences lies above
    the smaller one, so only the larger jump separates classes."""
    t = [10.0] * 100 + [12.0] * 100 + [30.0] * 100
    lab, bounds = orules.labels(t)
    assert bounds == [200]
    assert lab == [0] * 200 + [1] * 100


def test_oracle_constant_times_one_class():
    lab, bounds = orules.labels([5.0] * 300)
    assert bounds == [] and set(lab) == {0}


# ------------------------------------------------------------ library == oracle

@pytest.mark.parametrize("n,seed", [(50, 1), (200, 2), (2016, 3), (2016, 4), (777, 5)])
def test_labels_match_oracle_on_integer_times(n, seed):
    rng = np.random.default_rng(seed)
    # clustered integer times: a few levels, integer noise (ties and flat
    # convolution stretches occur)
    levels = rng.choice([100, 130, 180, 260], size=n, p=[0.4, 0.3, 0.2, 0.1])
    t = (levels + rng.integers(0, 6, size=n)).astype(np.float64)
    got = rules.class_labels(t)
    lab, bounds = orules.labels(t.tolist())
    assert got["labels"].tolist() == lab
    assert got["bounds"].tolist() == bounds
    assert got["radius"] == orules.radius(n)


def test_conv_matches_oracle():
    a = np.sort(np.random.default_rng(9).integers(0, 1000, 301)).astype(np.float64)
    for r in (1, 2, 7):
        c, _ = orules.step_conv(a.tolist(), r)
        assert rules.step_convolution(a, r).tolist() == c


def _timing_like(n, seed):
    """Float times shaped like a plan sweep: a few levels 45-100 us apart by
    uneven steps, with noise of about a microsecond (no sum is exact)."""
    rng = np.random.default_rng(seed)
    levels = rng.choice([45.3e-6, 52.1e-6, 71.7e-6, 98.9e-6], size=n, p=[0.1, 0.3, 0.5, 0.1])
    return levels + rng.normal(0.0, 1.1e-6, size=n) + rng.random(n) * 1e-7


@pytest.mark.parametrize("n,seed", [(50, 11), (400, 12), (2016, 13), (2016, 14)])
def test_conv_and_labels_match_oracle_on_float_times(n, seed):
    """On measured-like float times the window sums are the same floating
    point expressions on both sides (bit-identical), so peaks, prominences,
    bounds and labels agree exactly."""
    t = _timing_like(n, seed)
    r = orules.radius(n)
    a = np.sort(t, kind="stable")
    c, _ = orules.step_conv(a.tolist(), r)
    got = rules.step_convolution(a, r)
    assert np.array_equal(got.view(np.int64), np.asarray(c, np.float64).view(np.int64))
    lab_lib = rules.class_labels(t)
    lab, bounds = orules.labels(t.tolist())
    assert lab_lib["bounds"].tolist() == bounds
    assert lab_lib["labels"].tolist() == lab


def test_features_match_oracle_full_space():
    space = rules.plan_space(4, 2)
    X, names = rules.features(space)
    keep = rules.varying(X)
    rows, onames = orules.pair_features(space)
    assert [n for n, k in zip(names, keep) if k] == onames
    assert X[:, keep].tolist() == rows


def test_varying_feature_count_closed_form():
    """Over the whole space, an ordering pair varies exactly when its two
    operations are on different chains of the DAG (start and end are fixed,
    each chain is totally ordered): 23 pairs; all three GPU pairs vary in
    stream (four canonical stream maps)."""
    space = rules.plan_space(4, 2)
    X, names = rules.features(space)
    kept = [n for n, k in zip(names, rules.varying(X)) if k]
    chains = [{"Pack", "CER-after-Pack", "CES-b4-PostSend", "PostSend", "WaitSend"},
              {"PostRecv", "WaitRecv", "yR"}, {"yL"}]
    n_cross = sum(len(a) * len(b) for i, a in enumerate(chains) for b in chains[i + 1:])
    assert n_cross == 23
    assert len([n for n in kept if " before " in n]) == n_cross
    assert len([n for n in kept if n.endswith("same stream")]) == 3


# ------------------------------------------------------------ tree, Alg. 1, rules

def test_alg1_trace():
    err = {2: .5, 3: .5, 4: .3, 5: .3, 6: .3, 7: .2}
    model, mln, hist = rules.search_leaves(lambda m: (err.get(m, .2), m))
    assert (model, mln) == (7, 7)
    assert [m for m, _ in hist] == [2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12]


def test_alg1_stops_after_five_sizes_without_gain():
    model, mln, hist = rules.search_leaves(lambda m: (0.4 if m < 9 else 0.1, m))
    assert mln == 2 and [m for m, _ in hist] == [2, 3, 4, 5, 6, 7]


def _rule_cost(space, seed=0):
    """Synthetic times decided by two design choices, as in the paper's
    fastest class: y_L on a different stream than Pack and y_L before the
    host wait for Pack.  Three levels with equal steps (the percentile rule
    keeps both boundaries only when their prominences tie) and a spread
    inside each level smaller than a step, shifted per seed."""
    rng = np.random.default_rng(seed)
    t = np.empty(len(space))
    for i, (order, s) in enumerate(space):
        fast_stream = s["Pack"] != s["yL"]
        early = order.index("yL") < order.index("CES-b4-PostSend")
        t[i] = 100.0 + (0 if fast_stream and early else 40 if fast_stream or early else 80)
    return t + float(rng.integers(0, 10))


def test_tree_recovers_rules_and_partitions_samples():
    space = rules.plan_space(4, 2)
    t = _rule_cost(space)
    dr = rules.design_rules(space, t)
    y = dr["labels"]["labels"]
    assert len(set(y.tolist())) == 3
    X, _ = rules.features(space, dr["all_names"])
    X = X[:, dr["mask"]]
    clf = dr["tree"]
    assert np.all(clf.predict(X) == y)                       # training error 0
    pred = clf.predict(X)
    for i in range(len(space)):                               # exactly one rule set fits
        fits = [r for r in dr["rules"] if rules.follows(X[i], r["conditions"])]
        assert len(fits) == 1 and fits[0]["class"] == pred[i]
    fastest = [r for r in dr["rules"] if r["class"] == 0]
    used = {c for r in fastest for c in r["text"]}
    assert "Pack, yL different streams" in used
    assert "yL before CES-b4-PostSend" in used
    assert sum(r["samples"] for r in dr["rules"]) == len(space)


def test_table_v_accuracy_full_space_is_one():
    space = rules.plan_space(4, 2)
    t = _rule_cost(space, 1)
    res = rules.class_accuracy(space, t, np.arange(len(space)))
    assert res["accuracy"] == 1.0 and res["n_classes"] == 3


def test_table_v_from_tree_search_subsets():
    space = rules.plan_space(4, 2)
    t = _rule_cost(space, 2)
    acc = {}
    for it in (50, 200, 2016):
        r = sp.spmv_mcts_run_table(4, t, iterations=it if it < 2016 else 0, seed=3)
        acc[it] = rules.class_accuracy(space, t, r["index"])["accuracy"]
    assert acc[2016] == 1.0
    assert all(0.0 <= a <= 1.0 for a in acc.values())
