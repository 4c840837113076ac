"""Design rules from benchmarked plans (Sec. IV of the paper).

The explored plans (from the exhaustive sweep or the tree search) and their
times become design rules in four steps:

* :func:`class_labels` -- sort the times, convolve them with a step kernel
  of radius r (0.5 % of the count, at least 1), keep the peaks of the
  convolution whose prominence reaches the 98th percentile of all peak
  prominences, and cut the sorted times into performance classes at those
  peaks (Sec. IV-A);
* :func:`features` -- one ordering bit per pair of operations (u before v)
  and one stream bit per pair of GPU operations (same stream), with the
  columns that never vary dropped (Sec. IV-B);
* :func:`fit_tree` -- CART (scikit-learn, gini, balanced class weights,
  max_depth = max_leaf_nodes - 1) with the leaf count chosen by Alg. 1
  (Sec. IV-C, Table IV);
* :func:`rules` -- every root-to-leaf path of the tree is one rule set for
  the class of its leaf (Sec. IV-D).

:func:`class_accuracy` is the experiment of Table V: classes and tree from a
subset of the space, applied to every plan, scored by the fraction whose
time falls inside the time range of the class it is put in.
"""
from __future__ import annotations

import itertools

import numpy as np

from . import (SPMV_N_VERTICES, SPMV_OP_PACK, SPMV_OP_YL, SPMV_OP_YR, spmv_op_name,
               spmv_plan_space_count, spmv_plan_space_get)

GPU_OPS = ("Pack", "yL", "yR")


# ------------------------------------------------------------------ plans

def plan_space(nranks: int = 4, n_streams: int = 2):
    """Every plan of the library's design space as (operation names in
    order, {GPU operation: canonical stream}), in index order."""
    out = []
    for i in range(spmv_plan_space_count(nranks, n_streams)):
        ops, smap = spmv_plan_space_get(nranks, n_streams, i)
        names = tuple(spmv_op_name(int(o)) for o in ops)
        streams = {spmv_op_name(v): int(smap[v]) for v in range(SPMV_N_VERTICES)
                   if smap[v] >= 0}
        out.append((names, streams))
    return out


# ------------------------------------------------------------------ labels

def step_radius(n: int) -> int:
    """Radius of the step kernel: 0.5 % of the measurements, at least 1."""
    return max(1, int(round(0.005 * n)))


def step_convolution(a_sorted: np.ndarray, r: int) -> np.ndarray:
    """c[j] = sum(a[j+r .. j+2r-1]) - sum(a[j .. j+r-1]) for every j where
    the kernel (r samples of -1, then r of +1) lies inside the array.
    c[j] measures the rise across the gap between sorted positions
    j + r - 1 and j + r."""
    a = np.asarray(a_sorted, np.float64)
    if a.size < 2 * r:
        return np.zeros(0)
    # Each window is summed in a fixed order: start from 0, add the r
    # samples after the gap left to right, then subtract the r samples up to
    # it left to right.  Every output is then the same floating-point
    # expression whatever the array length, so measured (non-integer) times
    # give reproducible peaks; an FFT or a library convolution may reorder
    # the additions and move a peak by one rounding.
    m = a.size - 2 * r + 1
    c = np.zeros(m)
    for k in range(r, 2 * r):
        c += a[k:k + m]
    for k in range(r):
        c -= a[k:k + m]
    return c


def class_labels(times, radius: int | None = None, percentile: float = 98.0) -> dict:
    """Performance classes of the measurements (0 = fastest).

    Returns {labels (per input, original order), bounds (sorted positions
    where a new class starts), conv, peaks (indices into conv), prominences,
    radius, order (argsort of times)}."""
    from scipy.signal import find_peaks
    t = np.asarray(times, np.float64)
    order = np.argsort(t, kind="stable")
    r = step_radius(t.size) if radius is None else int(radius)
    conv = step_convolution(t[order], r)
    peaks, props = find_peaks(conv, prominence=(None, None))
    prom = props["prominences"] if peaks.size else np.zeros(0)
    if peaks.size:
        keep = prom >= np.percentile(prom, percentile)
        peaks, prom = peaks[keep], prom[keep]
    bounds = np.sort(peaks + r)                 # first sorted position of the next class
    lab_sorted = np.searchsorted(bounds, np.arange(t.size), side="right")
    labels = np.empty(t.size, np.int64)
    labels[order] = lab_sorted
    return {"labels": labels, "bounds": bounds, "conv": conv, "peaks": peaks,
            "prominences": prom, "radius": r, "order": order}


# ------------------------------------------------------------------ features

def feature_names(plans):
    """Names of every pairwise feature over the operations of the plans:
    'u before v' for each unordered pair (u, v) of operations, u ahead of v
    in the first plan, and 'u, v same stream' for each pair of GPU
    operations."""
    ops = list(plans[0][0])
    names = [f"{u} before {v}" for u, v in itertools.combinations(ops, 2)]
    gpu = [g for g in GPU_OPS if g in ops]
    names += [f"{u}, {v} same stream" for u, v in itertools.combinations(gpu, 2)]
    return names


def features(plans, names=None):
    """Feature matrix (uint8, one row per plan) over ``names`` (default:
    :func:`feature_names`)."""
    names = feature_names(plans) if names is None else names
    X = np.zeros((len(plans), len(names)), np.uint8)
    for j, nm in enumerate(names):
        if nm.endswith(" same stream"):
            u, v = nm[:-len(" same stream")].split(", ")
            X[:, j] = [s[u] == s[v] for _, s in plans]
        else:
            u, v = nm.split(" before ")
            X[:, j] = [o.index(u) < o.index(v) for o, _ in plans]
    return X, list(names)


def varying(X) -> np.ndarray:
    """Mask of the columns that take both values (constant columns carry no
    information and are removed)."""
    X = np.asarray(X)
    if X.shape[0] == 0:
        return np.zeros(X.shape[1], bool)
    return (X != X[0]).any(axis=0)


# ------------------------------------------------------------------ tree

def train(X, y, max_leaf_nodes: int, seed: int = 0):
    """CART with the parameters of Table IV; returns (training error,
    classifier)."""
    from sklearn.tree import DecisionTreeClassifier
    clf = DecisionTreeClassifier(criterion="gini", class_weight="balanced",
                                 max_leaf_nodes=max_leaf_nodes,
                                 max_depth=max(1, max_leaf_nodes - 1), random_state=seed)
    clf.fit(X, y)
    err = float(np.mean(clf.predict(X) != y))
    return err, clf


def search_leaves(train_fn, start: int = 2, tries: int = 5):
    """Alg. 1: grow max_leaf_nodes from ``start`` while the training error
    shrinks, looking up to ``tries`` sizes ahead each round.  ``train_fn(mln)``
    returns (error, model).  Returns (model, mln, history [(mln, error)])."""
    mln = start
    cur, model = train_fn(mln)
    history = [(mln, cur)]
    err = np.inf
    while cur < err:
        err = cur
        for i in range(1, tries + 1):
            c, m = train_fn(mln + i)
            history.append((mln + i, c))
            if c < err:
                cur, model, mln = c, m, mln + i
                break
    return model, mln, history


def fit_tree(X, y, seed: int = 0):
    """Alg. 1 over :func:`train`.  Returns (classifier, max_leaf_nodes,
    history [(mln, error, depth)])."""
    depth = {}

    def fn(mln):
        e, clf = train(X, y, mln, seed)
        depth[mln] = clf.get_depth()
        return e, clf
    clf, mln, hist = search_leaves(fn)
    return clf, mln, [(m, e, depth[m]) for m, e in hist]


# ------------------------------------------------------------------ rules

def _condition(name: str, value: bool) -> str:
    if name.endswith(" same stream"):
        u, v = name[:-len(" same stream")].split(", ")
        return f"{u}, {v} {'same stream' if value else 'different streams'}"
    u, v = name.split(" before ")
    return f"{u} before {v}" if value else f"{v} before {u}"


def rules(clf, names):
    """Every root-to-leaf path of the tree: {class, samples, counts (per
    class), leaf, conditions [(feature, value)], text [...]}, sorted by class
    then by samples (most first)."""
    tr = clf.tree_
    out = []

    def walk(node, conds):
        if tr.children_left[node] == tr.children_right[node]:       # leaf
            counts = tr.value[node][0]
            out.append({"leaf": int(node), "class": int(clf.classes_[int(np.argmax(counts))]),
                        "samples": int(tr.n_node_samples[node]),
                        "conditions": list(conds),
                        "text": [_condition(names[f], v) for f, v in conds]})
            return
        f = int(tr.feature[node])          # binary feature: <= 0.5 means 0
        walk(int(tr.children_left[node]), conds + [(f, False)])
        walk(int(tr.children_right[node]), conds + [(f, True)])

    walk(0, [])
    out.sort(key=lambda d: (d["class"], -d["samples"]))
    return out


def follows(X_row, conditions) -> bool:
    return all(bool(X_row[f]) == v for f, v in conditions)


# ------------------------------------------------------------------ Table V

def design_rules(plans, times, seed: int = 0) -> dict:
    """Labels, features, tree and rule sets for explored plans."""
    lab = class_labels(times)
    X_all, names = features(plans)
    keep = varying(X_all)
    X = X_all[:, keep]
    kept = [n for n, k in zip(names, keep) if k]
    y = lab["labels"]
    if len(np.unique(y)) < 2:
        return {"labels": lab, "names": kept, "mask": keep, "all_names": names, "tree": None,
                "rules": [], "mln": 1, "history": []}
    clf, mln, hist = fit_tree(X, y, seed)
    return {"labels": lab, "names": kept, "mask": keep, "all_names": names, "tree": clf,
            "rules": rules(clf, kept), "mln": mln, "history": hist}


def class_accuracy(space, all_times, subset, seed: int = 0) -> dict:
    """Table V: classes and tree from the plans ``subset`` (indices into
    ``space``) and their times; every plan of ``space`` is classified by the
    tree and counted correct when its time lies within [fastest, slowest] of
    the subset's samples of that class."""
    all_times = np.asarray(all_times, np.float64)
    subset = np.asarray(subset, np.int64)
    plans = [space[i] for i in subset]
    t_sub = all_times[subset]
    dr = design_rules(plans, t_sub, seed)
    y = dr["labels"]["labels"]
    ranges = {int(c): (float(t_sub[y == c].min()), float(t_sub[y == c].max()))
              for c in np.unique(y)}
    if dr["tree"] is None:
        pred = np.zeros(len(space), np.int64)
    else:
        X_all, _ = features(space, dr["all_names"])
        pred = dr["tree"].predict(X_all[:, dr["mask"]])
    lo = np.array([ranges[int(c)][0] for c in pred])
    hi = np.array([ranges[int(c)][1] for c in pred])
    ok = (all_times >= lo) & (all_times <= hi)
    return {"accuracy": float(ok.mean()), "n_classes": len(ranges), "ranges": ranges,
            "leaves": dr["mln"], "depth": int(dr["tree"].get_depth()) if dr["tree"] else 0,
            "rules": dr["rules"]}
