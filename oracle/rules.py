"""Class labels and feature vectors of Sec. IV -- TEST INFRASTRUCTURE.

Plain loops over the definitions, used only by the tests to check the
library's rule generation (which uses numpy's convolution and scipy's peak
finder).  Shares no code with the library.

* :func:`step_conv` -- the sorted times convolved with the step kernel of
  Sec. IV-A, only where the kernel lies fully inside the data.  The printed
  kernel and summation ranges do not agree on its support; the reading taken
  is r samples of -1 (m = -r+1 .. 0) followed by r samples of +1
  (m = 1 .. r), so c_i = sum_{m=1..r} a_{i+m} - sum_{m=-r+1..0} a_{i+m}.
* :func:`local_peaks` -- samples larger than both neighbours; a flat top
  (equal samples bounded by smaller ones) counts once, at its middle sample
  (rounded down), as in the peak finder the paper cites.
* :func:`prominence` -- height of a peak above the higher of the lowest
  points reached walking left and right until a strictly higher sample or
  the end of the data.
* :func:`labels` -- peaks whose prominence reaches the 98th percentile of
  all prominences (at least the top peak is kept) become class boundaries.
* :func:`pair_features` -- ordering bit per operation pair, same-stream bit
  per pair of GPU operations (Sec. IV-B), with constant columns dropped.
"""
from __future__ import annotations

import numpy as np


def radius(n: int) -> int:
    """0.5 % of the number of measurements, at least 1 (Sec. IV-A)."""
    return max(1, int(round(0.005 * n)))


def step_conv(a, r: int):
    """Values c_i for i = r-1 .. len(a)-r-1 (the kernel inside the data);
    returns (list of c_i, first i)."""
    a = [float(v) for v in a]
    out = []
    for i in range(r - 1, len(a) - r):
        s = 0.0
        for m in range(1, r + 1):
            s += a[i + m]
        for m in range(-r + 1, 1):
            s -= a[i + m]
        out.append(s)
    return out, r - 1


def local_peaks(x):
    peaks = []
    i = 1
    n = len(x)
    while i < n - 1:
        if x[i - 1] < x[i]:
            j = i
            while j + 1 < n and x[j + 1] == x[i]:
                j += 1
            if j + 1 < n and x[j + 1] < x[i]:
                peaks.append((i + j) // 2)
                i = j + 1
                continue
            i = j + 1
            continue
        i += 1
    return peaks


def prominence(x, p: int) -> float:
    h = x[p]
    left_min = h
    i = p
    while i > 0 and x[i - 1] <= h:
        i -= 1
        left_min = min(left_min, x[i])
    right_min = h
    i = p
    while i < len(x) - 1 and x[i + 1] <= h:
        i += 1
        right_min = min(right_min, x[i])
    return h - max(left_min, right_min)


def labels(times, r: int | None = None, percentile: float = 98.0):
    """Class of each measurement (0 = fastest), in input order, and the
    sorted positions where each class after the first begins."""
    t = list(times)
    order = sorted(range(len(t)), key=lambda k: (t[k], k))
    a = [t[k] for k in order]
    r = radius(len(a)) if r is None else r
    conv, first = step_conv(a, r)
    peaks = local_peaks(conv)
    bounds = []
    if peaks:
        prom = [prominence(conv, p) for p in peaks]
        cut = np.percentile(prom, percentile)
        # c_i spans the gap between sorted positions i and i + 1
        bounds = sorted(first + p + 1 for p, q in zip(peaks, prom) if q >= cut)
    lab = [0] * len(t)
    for pos, k in enumerate(order):
        lab[k] = sum(1 for b in bounds if b <= pos)
    return lab, bounds


def pair_features(plans, gpu_ops=("Pack", "yL", "yR")):
    """plans: list of (ordered operation names, {GPU op: stream}).  Returns
    (rows of 0/1, names) with the constant columns removed; names read
    'u before v' (u ahead of v in the first plan) and 'u, v same stream'."""
    ops = list(plans[0][0])
    names, cols = [], []
    for a in range(len(ops)):
        for b in range(a + 1, len(ops)):
            u, v = ops[a], ops[b]
            names.append(f"{u} before {v}")
            cols.append([1 if o.index(u) < o.index(v) else 0 for o, _ in plans])
    gpu = [g for g in gpu_ops if g in ops]
    for a in range(len(gpu)):
        for b in range(a + 1, len(gpu)):
            u, v = gpu[a], gpu[b]
            names.append(f"{u}, {v} same stream")
            cols.append([1 if s[u] == s[v] else 0 for _, s in plans])
    keep = [j for j, c in enumerate(cols) if min(c) != max(c)]
    rows = [[cols[j][i] for j in keep] for i in range(len(plans))]
    return rows, [names[j] for j in keep]
