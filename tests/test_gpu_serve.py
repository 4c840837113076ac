"""Serving: resident matrices, HBM-budget admission, continuous batching.

Each request's y must be bit-identical whether it is served alone (the plain
per-call mode) or batched with others, and within tolerance of the oracle;
the budget must bound the device bytes in use."""
import numpy as np
import pytest

import gen
import oracle
import paper_2203_02530_amd as sp
from gpu_util import bits, log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch
    assert torch.cuda.is_available()
    oracle.build(force=False)
    yield


def _pool(k=6, seed=0):
    rng = np.random.default_rng(seed)
    sizes = np.rint(10 ** rng.uniform(3, 4.5, k)).astype(int)
    return [gen.banded_random(int(n), seed=5000 + i) for i, n in enumerate(sizes)]


def _trace(mats, n_req, rate, seed):
    import torch
    rng = np.random.default_rng(seed)
    arr = np.cumsum(rng.exponential(1.0 / rate, n_req))
    ids = rng.integers(0, len(mats), n_req).astype(np.int32)
    xs, ys, xnp = [], [], []
    for i in range(n_req):
        n = mats[ids[i]].n_rows
        x = gen.x_normal(n, 5300 + i)
        xnp.append(x)
        xs.append(torch.from_numpy(x).pin_memory())
        ys.append(torch.full((n,), float("nan"), dtype=torch.float64).pin_memory())
    return arr - arr[0], ids, xs, ys, xnp


def _serve(mats, arr, ids, xs, ys, opts):
    srv = sp.spmv_server_create(opts)
    try:
        for A in mats:
            sp.spmv_server_add_matrix(srv, A)
        sp.spmv_server_start(srv)
        lat, wall = sp.spmv_server_run_trace(srv, ids, arr, xs, ys)
        st = sp.spmv_server_stats(srv)
    finally:
        sp.spmv_server_destroy(srv)
    return lat, wall, st, [y.numpy().copy() for y in ys]


def test_batched_equals_plain_and_oracle():
    mats = _pool()
    arr, ids, xs, ys, xnp = _trace(mats, 300, 20000.0, 1)
    log("serve batched")
    lat_b, wall_b, st_b, y_b = _serve(mats, arr, ids, xs, ys, {"mode": 0})
    for y in ys:
        y.fill_(float("nan"))
    log("serve plain")
    lat_p, wall_p, st_p, y_p = _serve(mats, arr, ids, xs, ys, {"mode": 1})
    assert st_b["completed"] == st_p["completed"] == 300
    assert st_p["mean_batch"] == 1.0 and st_p["peak_inflight"] == 1
    assert st_b["mean_batch"] >= 1.0
    assert np.all(lat_b > 0) and np.all(lat_p > 0)
    for i in range(300):
        assert np.array_equal(bits(y_b[i]), bits(y_p[i])), i
    # oracle parity on every request
    for i in range(300):
        A = mats[ids[i]]
        ref, ax = oracle.spmv_dot2(A.row_ptr, A.col_idx, A.val, xnp[i])
        assert oracle.within_tolerance(y_b[i], ref, ax).all(), i


def test_large_batches_copy_descriptors():
    """Batches of at most eight requests take their descriptors in the kernel
    arguments, larger ones copy them to the device first: 256 requests that
    arrive at once make batches of up to 64 (the copied form), the plain mode
    serves each alone (the inline form), and both agree bit for bit and with
    the oracle."""
    mats = _pool(k=8, seed=2)
    arr, ids, xs, ys, xnp = _trace(mats, 256, 1e9, 4)
    log("serve large batches")
    _, _, st_b, y_b = _serve(mats, arr, ids, xs, ys, {"mode": 0, "max_batch": 64})
    for y in ys:
        y.fill_(float("nan"))
    log("serve large batches, plain")
    _, _, st_p, y_p = _serve(mats, arr, ids, xs, ys, {"mode": 1})
    assert st_b["completed"] == st_p["completed"] == 256
    assert st_b["mean_batch"] > 8.0, st_b
    for i in range(256):
        assert np.array_equal(bits(y_b[i]), bits(y_p[i])), i
        A = mats[ids[i]]
        ref, ax = oracle.spmv_dot2(A.row_ptr, A.col_idx, A.val, xnp[i])
        assert oracle.within_tolerance(y_b[i], ref, ax).all(), i


def test_largest_pool_matrices():
    """The largest matrices of the serving pool's recipe (10^6 and 3*10^5
    rows, 5..27 entries per row in half-bandwidth 2000) at full size: 40
    requests arriving at once, batched and plain bit-identical, every
    request within tolerance of the oracle."""
    mats = [gen.banded_random(1_000_000, seed=5001), gen.banded_random(300_000, seed=5002)]
    arr, ids, xs, ys, xnp = _trace(mats, 40, 1e9, 3)
    log("serve largest batched")
    _, _, st_b, y_b = _serve(mats, arr, ids, xs, ys, {"mode": 0})
    for y in ys:
        y.fill_(float("nan"))
    log("serve largest plain")
    _, _, st_p, y_p = _serve(mats, arr, ids, xs, ys, {"mode": 1})
    assert st_b["completed"] == st_p["completed"] == 40
    assert st_b["mean_batch"] > 1.0
    for i in range(40):
        assert np.array_equal(bits(y_b[i]), bits(y_p[i])), i
        A = mats[ids[i]]
        ref, ax = oracle.spmv_dot2(A.row_ptr, A.col_idx, A.val, xnp[i])
        assert oracle.within_tolerance(y_b[i], ref, ax).all(), i


def test_budget_bounds_device_bytes():
    """A budget that fits the matrices plus only a few requests at a time:
    all requests still complete, and buffers in use never exceed the room."""
    import torch
    mats = _pool(4, seed=3)
    arr, ids, xs, ys, xnp = _trace(mats, 120, 50000.0, 2)
    # resident size from a generous server, then a tight one
    srv = sp.spmv_server_create({})
    try:
        for A in mats:
            sp.spmv_server_add_matrix(srv, A)
        resident = sp.spmv_server_stats(srv)["resident_bytes"]
    finally:
        sp.spmv_server_destroy(srv)
    largest = max(2 * (((max(A.n_rows, 1) * 8) + 255) // 256 * 256) for A in mats)
    budget = resident + 4 * 4 * 2 * 256 + 3 * largest + (1 << 20)   # stage buffers + 3 requests
    lat, wall, st, y = _serve(mats, arr, ids, xs, ys, {"budget_bytes": budget})
    assert st["completed"] == 120
    assert st["resident_bytes"] + st["peak_inflight_bytes"] <= budget
    for i in range(120):
        A = mats[ids[i]]
        ref, ax = oracle.spmv_dot2(A.row_ptr, A.col_idx, A.val, xnp[i])
        assert oracle.within_tolerance(y[i], ref, ax).all(), i


def test_budget_rejections():
    A = gen.banded_random(20000, seed=7)
    srv = sp.spmv_server_create({"budget_bytes": 1 << 20})     # 1 MiB: matrix does not fit
    try:
        with pytest.raises(sp.SpmvError) as e:
            sp.spmv_server_add_matrix(srv, A)
        assert e.value.code == sp.SPMV_EBUDGET
    finally:
        sp.spmv_server_destroy(srv)


def test_create_destroy_returns_device_memory():
    """Every device allocation of a server (request arena, per-slot stage
    descriptors, resident plans) is released by destroy: free device memory
    returns to its level after repeated create / start / destroy cycles."""
    import torch
    A = gen.banded_random(5000, seed=8)

    def cycle():
        srv = sp.spmv_server_create({"max_epochs": 32, "max_inflight": 4})
        try:
            sp.spmv_server_add_matrix(srv, A)
            sp.spmv_server_start(srv)
        finally:
            sp.spmv_server_destroy(srv)

    cycle()                                   # runtime pools warm up
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    for _ in range(16):
        cycle()
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    # 16 cycles x 32 slots of descriptor buffers would be >= 512 allocations
    assert free0 - free1 <= (2 << 20), (free0, free1)
