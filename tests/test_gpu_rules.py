"""Design rules (Sec. IV) on times measured on the device.

The plan times of a real sweep are floats with timing noise, the input on
which a different summation order in the label convolution could move a
peak.  A small share's whole plan space is timed on the GPU, and the
library's labels, class bounds and feature rows must equal the oracle's
plain-loop definitions on exactly those times."""
import numpy as np
import pytest

import gen
from oracle import rules as orules
from paper_2203_02530_amd import rules, tune
from gpu_util import log

pytestmark = pytest.mark.gpu


def test_rules_on_device_timed_sweep_match_oracle():
    import torch
    assert torch.cuda.is_available()
    A = gen.laplacian_3d7(32)
    x = gen.x_uniform(A.n_cols, 2)
    P, r = 4, 1
    log("sweep of 2016 plans, 3D 7-point 32^3 P=4 r=1")
    res = tune.sweep_plans(A, P, r, x, 2, None, t_measure=0.002, n_measure=1)
    t = np.empty(len(res))
    for d in res:
        t[d["index"]] = d["t"]
    assert t.size == 2016 and np.all(t > 0)
    # measured times: non-integer, with ties unlikely
    assert np.unique(t).size > 1000

    got = rules.class_labels(t)
    lab, bounds = orules.labels(t.tolist())
    assert got["bounds"].tolist() == bounds
    assert got["labels"].tolist() == lab
    a = np.sort(t, kind="stable")
    c, _ = orules.step_conv(a.tolist(), got["radius"])
    assert np.array_equal(got["conv"].view(np.int64), np.asarray(c, np.float64).view(np.int64))

    # feature rows over the whole space, and over a tree-search subset as the
    # Table V experiment trains on
    space = rules.plan_space(P, 2)
    X, names = rules.features(space)
    keep = rules.varying(X)
    rows, onames = orules.pair_features(space)
    assert [n for n, k in zip(names, keep) if k] == onames
    assert X[:, keep].tolist() == rows
    import paper_2203_02530_amd as sp
    sub = sp.spmv_mcts_run_table(P, t, iterations=200, seed=1)["index"]
    sub_plans = [space[i] for i in sub]
    Xs, ns = rules.features(sub_plans)
    ks = rules.varying(Xs)
    rows_s, onames_s = orules.pair_features(sub_plans)
    assert [n for n, k in zip(ns, ks) if k] == onames_s
    assert Xs[:, ks].tolist() == rows_s
    lab_s = rules.class_labels(t[sub])
    lab_o, bounds_o = orules.labels(t[sub].tolist())
    assert lab_s["labels"].tolist() == lab_o and lab_s["bounds"].tolist() == bounds_o
