"""Seeded synthetic inputs for the row-partitioned SpMV.

This module only builds matrices and vectors: sparsity patterns, values and
right-hand sides drawn from fixed seeds.  It holds none of the SpMV
arithmetic, so both the CPU oracle (``oracle/``) and the HIP path
(``paper_2203_02530_amd``) can take their inputs from it without sharing any
part of the method.

Every matrix is returned as a :class:`CSR` with int32 ``row_ptr``/``col_idx``,
float64 ``val``, column indices strictly ascending inside each row.

Workloads (the paper's own input is the banded matrix of Sec. III, the only
input it measures; the others are the stencil, power-law and serving
workloads the port is measured on):

* :func:`laplacian_2d5`  -- 2D 5-point Laplacian, diag 4, off -1.
* :func:`laplacian_3d7`  -- 3D 7-point Laplacian, diag 6, off -1.
* :func:`stencil_3d27`   -- 3D 27-point stencil, off-diagonals U(0,1],
  diagonal = sum of the row's off-diagonals + 1.
* :func:`banded_uniform` -- the paper's banded matrix (Sec. III): a fixed
  number of distinct columns per row drawn uniformly inside the band
  ``|i - j| <= half_bw``, values N(0,1).
* :func:`power_law`      -- lognormal row lengths, uniform distinct columns.
* :func:`banded_random`  -- per-row length uniform in [lo, hi], columns
  distinct inside ``|i - j| <= half_bw`` (serving pool).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = [
    "CSR", "laplacian_2d5", "laplacian_3d7", "stencil_3d27", "banded_uniform",
    "power_law", "power_law_share", "banded_random", "x_uniform", "x_normal", "x_integer",
    "sine_mode", "WORKLOADS", "workload",
]


@dataclass
class CSR:
    n_rows: int
    n_cols: int
    row_ptr: np.ndarray  # int32 [n_rows + 1]
    col_idx: np.ndarray  # int32 [nnz]
    val: np.ndarray      # float64 [nnz]

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def check(self) -> None:
        """Structural sanity of a generated matrix (not part of the method)."""
        rp, ci = self.row_ptr, self.col_idx
        assert rp.dtype == np.int32 and ci.dtype == np.int32
        assert self.val.dtype == np.float64
        assert rp[0] == 0 and rp[-1] == ci.size == self.val.size
        assert np.all(np.diff(rp) >= 0)
        if ci.size:
            assert ci.min() >= 0 and ci.max() < self.n_cols
            d = np.diff(ci.astype(np.int64))
            row_start = np.zeros(ci.size, bool)
            row_start[rp[:-1][np.diff(rp) > 0]] = True
            # inside a row, columns strictly ascend
            assert np.all((d > 0) | row_start[1:])


def _csr_from_mask(cols: np.ndarray, valid: np.ndarray, vals: np.ndarray,
                   n_cols: int) -> CSR:
    counts = valid.sum(axis=1, dtype=np.int64)
    row_ptr = np.zeros(cols.shape[0] + 1, np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    if row_ptr[-1] >= 2**31:
        raise ValueError("nnz does not fit int32")
    return CSR(cols.shape[0], n_cols, row_ptr.astype(np.int32),
               np.ascontiguousarray(cols[valid], dtype=np.int32),
               np.ascontiguousarray(vals[valid], dtype=np.float64))


def _stencil(shape: tuple[int, ...], radius_offsets: list[tuple[int, ...]]):
    """Column pattern of a stencil on a row-major grid.

    Offsets are sorted so that the flat column offset ascends, which keeps the
    columns of every row in ascending order.  Returns (cols, valid, is_diag).
    """
    n = int(np.prod(shape))
    strides = [int(np.prod(shape[d + 1:])) for d in range(len(shape))]
    offs = sorted(radius_offsets, key=lambda o: sum(o[d] * strides[d] for d in range(len(shape))))
    coords = [c.reshape(-1) for c in np.indices(shape, dtype=np.int32)]
    flat = np.arange(n, dtype=np.int64)
    k = len(offs)
    cols = np.empty((n, k), np.int32)
    valid = np.empty((n, k), bool)
    is_diag = np.zeros(k, bool)
    for j, off in enumerate(offs):
        ok = np.ones(n, bool)
        for d, o in enumerate(off):
            if o:
                ok &= (coords[d] + o >= 0) & (coords[d] + o < shape[d])
        delta = sum(off[d] * strides[d] for d in range(len(shape)))
        cols[:, j] = np.where(ok, flat + delta, 0)
        valid[:, j] = ok
        is_diag[j] = all(o == 0 for o in off)
    return cols, valid, is_diag


def laplacian_2d5(nx: int, ny: int | None = None) -> CSR:
    """2D 5-point Laplacian on an ny x nx grid (row index = y*nx + x)."""
    ny = nx if ny is None else ny
    offs = [(0, 0), (-1, 0), (1, 0), (0, -1), (0, 1)]
    cols, valid, is_diag = _stencil((ny, nx), offs)
    vals = np.where(is_diag[None, :], 4.0, -1.0) * np.ones_like(cols, dtype=np.float64)
    return _csr_from_mask(cols, valid, vals, nx * ny)


def laplacian_3d7(n: int) -> CSR:
    """3D 7-point Laplacian on an n^3 grid (row index = (z*n + y)*n + x)."""
    offs = [(0, 0, 0), (-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1)]
    cols, valid, is_diag = _stencil((n, n, n), offs)
    vals = np.where(is_diag[None, :], 6.0, -1.0) * np.ones_like(cols, dtype=np.float64)
    return _csr_from_mask(cols, valid, vals, n ** 3)


def stencil_3d27(n: int, seed: int = 3) -> CSR:
    """3D 27-point stencil: off-diagonals U(0,1], diagonal = their row sum + 1."""
    offs = [(a, b, c) for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1)]
    cols, valid, is_diag = _stencil((n, n, n), offs)
    rng = np.random.default_rng(seed)
    vals = 1.0 - rng.random(cols.shape)          # (0, 1]
    vals[:, is_diag] = 0.0
    vals[~valid] = 0.0
    vals[:, is_diag] = vals.sum(axis=1, keepdims=True) + 1.0
    return _csr_from_mask(cols, valid, vals, n ** 3)


def _distinct_sorted_rows(rng, lo: np.ndarray, hi: np.ndarray, lengths: np.ndarray,
                          n_cols: int) -> np.ndarray:
    """Per row i, ``lengths[i]`` distinct columns uniform in [lo[i], hi[i]],
    concatenated row by row in ascending order.

    Sorted uniforms come directly as order statistics: with E_1..E_{L+1}
    i.i.d. exponential, (E_1 + .. + E_j) / (E_1 + .. + E_{L+1}), j = 1..L, are
    L sorted U(0,1) draws, so no sort is needed.  A row whose floored columns
    collide (rare) is redrawn without replacement.
    """
    n = lengths.size
    total = int(lengths.sum())
    if total == 0:
        return np.zeros(0, np.int64)
    seg = lengths + 1                                   # L + 1 spacings per row
    e = rng.standard_exponential(int(seg.sum()))
    c = np.cumsum(e)
    ends = np.cumsum(seg) - 1                           # index of each row's last spacing
    starts = ends - lengths                             # first spacing of each row
    before = np.where(starts > 0, c[starts - 1], 0.0)   # cumsum before the row
    tot = c[ends] - before
    row = np.repeat(np.arange(n, dtype=np.int64), lengths)
    # positions of the first L partial sums of each row inside c
    keep = np.ones(c.size, bool)
    keep[ends] = False
    u = c[keep]
    u -= before[row]
    u /= tot[row]
    if np.all(lo == lo[0]) and np.all(hi == hi[0]):      # one common range
        width = int(hi[0] - lo[0] + 1)
        cols = np.minimum((u * width).astype(np.int64), width - 1)
        cols += int(lo[0])
    else:
        width = (hi - lo + 1)[row]
        cols = lo[row] + np.minimum((u * width).astype(np.int64), width - 1)
    dup = np.zeros(total, bool)
    dup[1:] = (cols[1:] == cols[:-1]) & (row[1:] == row[:-1])
    if dup.any():
        offs = np.zeros(n + 1, np.int64)
        np.cumsum(lengths, out=offs[1:])
        for r in np.unique(row[dup]):
            a, b = offs[r], offs[r + 1]
            cols[a:b] = np.sort(lo[r] + rng.choice(int(hi[r] - lo[r] + 1), size=int(b - a),
                                                   replace=False))
    return cols


def banded_uniform(n: int = 150_000, per_row: int = 10, half_bw: int = 37_500,
                   seed: int = 100) -> CSR:
    """The paper's banded matrix (Sec. III): ``per_row`` distinct columns per row,
    uniform inside ``|i - j| <= half_bw`` (clipped to the matrix), values N(0,1).

    The paper gives 150,000 rows, 1,500,000 non-zeros and bandwidth 150000/4;
    the bandwidth is read as the half-width ``|i - j| <= n/4``.
    """
    rng = np.random.default_rng(seed)
    i = np.arange(n, dtype=np.int64)
    lo = np.maximum(i - half_bw, 0)
    hi = np.minimum(i + half_bw, n - 1)
    lengths = np.minimum(np.full(n, per_row, np.int64), hi - lo + 1)
    cols = _distinct_sorted_rows(rng, lo, hi, lengths, n)
    row_ptr = np.zeros(n + 1, np.int64)
    np.cumsum(lengths, out=row_ptr[1:])
    val = rng.standard_normal(cols.size)
    return CSR(n, n, row_ptr.astype(np.int32), cols.astype(np.int32), val)


def power_law(n: int = 4_000_000, mean_len: float = 16.0, sigma: float = 1.2,
              max_len: int = 10_000, seed: int = 4000) -> CSR:
    """Row lengths rint(lognormal) with arithmetic mean ``mean_len`` (so
    mu = ln(mean_len) - sigma^2/2), clipped to [1, max_len]; columns distinct and
    uniform over [0, n); values N(0,1)."""
    rng = np.random.default_rng(seed)
    mu = math.log(mean_len) - 0.5 * sigma * sigma
    lengths = np.rint(rng.lognormal(mu, sigma, n)).astype(np.int64)
    lengths = np.clip(lengths, 1, min(max_len, n))
    lo = np.zeros(n, np.int64)
    hi = np.full(n, n - 1, np.int64)
    cols = _distinct_sorted_rows(rng, lo, hi, lengths, n)
    row_ptr = np.zeros(n + 1, np.int64)
    np.cumsum(lengths, out=row_ptr[1:])
    if row_ptr[-1] >= 2**31:
        raise ValueError("nnz does not fit int32")
    val = rng.standard_normal(cols.size)
    return CSR(n, n, row_ptr.astype(np.int32), cols.astype(np.int32), val)


def power_law_share(n: int = 4_000_000, nranks: int = 16, rank: int = 5,
                    mean_len: float = 16.0, sigma: float = 1.2, max_len: int = 10_000,
                    seed: int = 4000) -> dict:
    """One rank's share of a power-law matrix, generated without the rest of
    the matrix: the rank's own rows in full (lengths, distinct uniform
    columns over [0, n), N(0,1) values), and, for every other rank q, the
    owned columns q's rows reference: q's entries land in this rank's column
    block with probability n_loc / n, so their count is binomial over q's
    total entries and the columns are uniform in the block (within-row
    distinctness of q's rows is not modelled).

    Returns dict(local=CSR with n_loc rows and global columns, lo, n_global,
    send_idx, send_off) -- the inputs of spmv_plan_create_local."""
    rng = np.random.default_rng(seed)
    mu = math.log(mean_len) - 0.5 * sigma * sigma
    lengths = np.clip(np.rint(rng.lognormal(mu, sigma, n)).astype(np.int64), 1, min(max_len, n))
    q = np.arange(nranks + 1, dtype=np.int64)
    blo = q * (n // nranks) + np.minimum(q, n % nranks)
    lo, hi = int(blo[rank]), int(blo[rank + 1])
    nl = hi - lo
    own = lengths[lo:hi]
    cols = _distinct_sorted_rows(rng, np.zeros(nl, np.int64), np.full(nl, n - 1, np.int64), own, n)
    row_ptr = np.zeros(nl + 1, np.int64)
    np.cumsum(own, out=row_ptr[1:])
    local = CSR(nl, n, row_ptr.astype(np.int32), cols.astype(np.int32),
                rng.standard_normal(cols.size))
    send, send_off = [], np.zeros(nranks + 1, np.int64)
    for qq in range(nranks):
        if qq == rank or nl == 0:
            idx = np.zeros(0, np.int64)
        else:
            tot = int(lengths[blo[qq]:blo[qq + 1]].sum())
            m = int(rng.binomial(tot, nl / n))
            idx = np.unique(rng.integers(0, nl, m))
        send.append(idx)
        send_off[qq + 1] = send_off[qq] + idx.size
    return dict(local=local, lo=lo, n_global=n, nranks=nranks, rank=rank,
                send_idx=np.concatenate(send).astype(np.int32), send_off=send_off.astype(np.int32))


def three_diagonals(n: int, d: int, seed: int = 0) -> CSR:
    """Rows with the columns i - d, i, i + d (those inside [0, n)), values
    N(0,1): offsets of exactly d from the row, for 16-bit boundary cases."""
    rng = np.random.default_rng(seed)
    i = np.arange(n)
    cols = np.stack([i - d, i, i + d], axis=1)
    valid = (cols >= 0) & (cols < n)
    counts = valid.sum(axis=1)
    rp = np.zeros(n + 1, np.int32)
    np.cumsum(counts, out=rp[1:])
    c = cols[valid].astype(np.int32)
    return CSR(n, n, rp, c, rng.standard_normal(c.size))


def banded_random(n: int, lo_len: int = 5, hi_len: int = 27, half_bw: int = 2000,
                  seed: int = 5000) -> CSR:
    """Row length uniform in {lo_len..hi_len}, columns distinct inside
    ``|i - j| <= half_bw`` (clipped), values N(0,1)."""
    rng = np.random.default_rng(seed)
    i = np.arange(n, dtype=np.int64)
    lo = np.maximum(i - half_bw, 0)
    hi = np.minimum(i + half_bw, n - 1)
    lengths = rng.integers(lo_len, hi_len + 1, n).astype(np.int64)
    lengths = np.minimum(lengths, hi - lo + 1)
    cols = _distinct_sorted_rows(rng, lo, hi, lengths, n)
    row_ptr = np.zeros(n + 1, np.int64)
    np.cumsum(lengths, out=row_ptr[1:])
    val = rng.standard_normal(cols.size)
    return CSR(n, n, row_ptr.astype(np.int32), cols.astype(np.int32), val)


def x_uniform(n: int, seed: int) -> np.ndarray:
    """x ~ U[-1, 1)."""
    return np.random.default_rng(seed).uniform(-1.0, 1.0, n)


def x_normal(n: int, seed: int) -> np.ndarray:
    """x ~ N(0, 1)."""
    return np.random.default_rng(seed).standard_normal(n)


def x_integer(n: int, seed: int, lo: int = -4, hi: int = 4) -> np.ndarray:
    """Small integer-valued x: every partial sum of an integer stencil row is exact."""
    return np.random.default_rng(seed).integers(lo, hi + 1, n).astype(np.float64)


def sine_mode(shape: tuple[int, ...], modes: tuple[int, ...]) -> np.ndarray:
    """prod_d sin(p_d * pi * (i_d + 1) / (N_d + 1)) on a row-major grid: a
    Dirichlet-Laplacian eigenvector used as a closed-form test vector."""
    v = np.ones(shape)
    for d, (nd, p) in enumerate(zip(shape, modes)):
        s = np.sin(p * math.pi * (np.arange(nd) + 1) / (nd + 1))
        sh = [1] * len(shape)
        sh[d] = nd
        v = v * s.reshape(sh)
    return v.reshape(-1)


# Named workloads: matrix builder, nranks, rank, x builder.  Sizes are the full
# measured sizes; tests scale them down through the ``small`` variants.
WORKLOADS = {
    "laplace2d_64": dict(build=lambda: laplacian_2d5(64), nranks=1, rank=0,
                         x=lambda n: x_uniform(n, 1),
                         desc="2D 5-point Laplacian 64x64, P=1"),
    "laplace3d_128_p4r1": dict(build=lambda: laplacian_3d7(128), nranks=4, rank=1,
                               x=lambda n: x_uniform(n, 2),
                               desc="3D 7-point Laplacian 128^3, P=4, rank 1 share"),
    "stencil27_150_p8r3": dict(build=lambda: stencil_3d27(150, seed=3), nranks=8, rank=3,
                               x=lambda n: x_normal(n, 30),
                               desc="3D 27-point stencil 150^3, P=8, rank 3 share"),
    "banded_150k_p4r1": dict(build=lambda: banded_uniform(150_000, 10, 37_500, seed=100),
                             nranks=4, rank=1, x=lambda n: x_normal(n, 101),
                             desc="banded 150000 rows, 10 nnz/row, half-bandwidth 37500, P=4, rank 1"),
    "powerlaw_4m_p16r5": dict(build=lambda: power_law(4_000_000, seed=4000), nranks=16, rank=5,
                              x=lambda n: x_normal(n, 4100),
                              desc="power-law 4M rows, lognormal(16,1.2), P=16, rank 5 share"),
}


def workload(name: str):
    w = WORKLOADS[name]
    A = w["build"]()
    return A, w["nranks"], w["rank"], w["x"](A.n_cols)
