"""CPU oracle for the row-partitioned distributed SpMV -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the HIP library
(``paper_2203_02530_amd``) and never imports it; inputs come from ``gen``.

Contents, each following the passage of the paper it cites:

* :func:`row_blocks` -- contiguous row blocks of A, x and y over P ranks
  (Sec. III-A: rows divided evenly across ranks; the first ``n mod P`` ranks
  take one extra row when P does not divide n).
* :func:`split` -- the rank's ``A = A_L + A_R`` split, the halo set ``x_R``
  and the per-destination send lists (Sec. III-A: A_L holds the columns of
  the locally held x entries, A_R the rest; each rank copies the x entries
  other ranks need into one buffer per destination).  Ordering conventions,
  where the paper is silent: halo columns ascending (hence grouped by owner
  in ascending rank order), send entries ascending per destination,
  destinations ascending.
* :func:`spmv_dot2` -- the plain CSR product, one compensated dot product per
  row (C, ``oracle.c``), plus ``|A||x|`` per row for the tolerance.
* :func:`share_reference` -- everything one rank's share of ``y = A x``
  produces: y, the local and remote partial products, the packed send buffer
  and the received halo.
* :func:`exact_rows` -- exact rational row products for tiny inputs.
* :func:`plan_space` -- the set of valid (operation order, stream map)
  implementations of the SpMV DAG (Sec. III-A, III-C2, Table III), by brute
  force over permutations.
"""
from __future__ import annotations

import ctypes
import itertools
import math
import os
import subprocess
from fractions import Fraction

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so (gcc, OpenMP, no FP contraction)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
               "-fno-fast-math", "-std=c99", "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        lib.orc_csr_dot2.argtypes = [ctypes.c_int64, P, P, P, P, P, P, ctypes.c_int]
        lib.orc_csr_dot2.restype = None
        lib.orc_csr_plain.argtypes = [ctypes.c_int64, P, P, P, P, P, ctypes.c_int]
        lib.orc_csr_plain.restype = None
        lib.orc_dot2.argtypes = [ctypes.c_int64, P, P]
        lib.orc_dot2.restype = ctypes.c_double
        lib.orc_num_threads.restype = ctypes.c_int
        lib.orc_set_threads.argtypes = [ctypes.c_int]
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def num_threads() -> int:
    return _load().orc_num_threads()


def set_threads(n: int) -> None:
    _load().orc_set_threads(n)


# ---------------------------------------------------------------- arithmetic

def dot2(a: np.ndarray, b: np.ndarray) -> float:
    """Compensated dot product of two dense FP64 vectors."""
    a = np.ascontiguousarray(a, np.float64)
    b = np.ascontiguousarray(b, np.float64)
    return _load().orc_dot2(a.size, _ptr(a), _ptr(b))


def spmv_dot2(row_ptr: np.ndarray, col_idx: np.ndarray, val: np.ndarray,
              x: np.ndarray, dynamic: bool = False):
    """Row products of a CSR block with x: returns (y, absax).

    ``row_ptr`` indexes ``col_idx``/``val`` directly (it may be a slice of a
    larger matrix's row pointer)."""
    row_ptr = np.ascontiguousarray(row_ptr, np.int32)
    col_idx = np.ascontiguousarray(col_idx, np.int32)
    val = np.ascontiguousarray(val, np.float64)
    x = np.ascontiguousarray(x, np.float64)
    n = row_ptr.size - 1
    y = np.empty(max(n, 0), np.float64)
    ax = np.empty(max(n, 0), np.float64)
    if n > 0:
        _load().orc_csr_dot2(n, _ptr(row_ptr), _ptr(col_idx), _ptr(val), _ptr(x),
                             _ptr(y), _ptr(ax), int(dynamic))
    return y, ax


def spmv_plain(row_ptr: np.ndarray, col_idx: np.ndarray, val: np.ndarray, x: np.ndarray,
               dynamic: bool = False) -> np.ndarray:
    """The plain (uncompensated) FP64 CSR product of a row block, OpenMP over
    rows: the CPU throughput baseline, not a reference."""
    row_ptr = np.ascontiguousarray(row_ptr, np.int32)
    col_idx = np.ascontiguousarray(col_idx, np.int32)
    val = np.ascontiguousarray(val, np.float64)
    x = np.ascontiguousarray(x, np.float64)
    n = row_ptr.size - 1
    y = np.empty(max(n, 0), np.float64)
    if n > 0:
        _load().orc_csr_plain(n, _ptr(row_ptr), _ptr(col_idx), _ptr(val), _ptr(x), _ptr(y),
                              int(dynamic))
    return y


# ---------------------------------------------------------------- partition

def row_blocks(n: int, P: int) -> np.ndarray:
    """lo[q] for q = 0..P: rank q owns rows [lo[q], lo[q+1]).

    ``lo_q = q * floor(n/P) + min(q, n mod P)``."""
    q = np.arange(P + 1, dtype=np.int64)
    return q * (n // P) + np.minimum(q, n % P)


def _split_rows(rp_rows, cols_all, vals_all, n: int, P: int, r: int) -> dict:
    """A_L / A_R / halo of rank r from its own rows (global column indices):
    rp_rows[0..n_loc] indexes cols_all / vals_all."""
    lo_all = row_blocks(n, P)
    lo, hi = int(lo_all[r]), int(lo_all[r + 1])
    n_loc = hi - lo
    grp = np.asarray(rp_rows, np.int64)
    b, e = grp[0], grp[-1]
    cols = np.asarray(cols_all[b:e], np.int64)
    vals = vals_all[b:e]
    row_of = np.repeat(np.arange(n_loc, dtype=np.int64), np.diff(grp))
    local = (cols >= lo) & (cols < hi)

    L_cnt = np.bincount(row_of[local], minlength=n_loc)
    L_ptr = np.zeros(n_loc + 1, np.int64)
    np.cumsum(L_cnt, out=L_ptr[1:])

    rem_cols = cols[~local]
    H = np.unique(rem_cols)
    recv_off = np.searchsorted(H, lo_all)          # owners are contiguous blocks
    rem_rows = row_of[~local]
    R_rows = np.unique(rem_rows)
    R_cnt = np.bincount(rem_rows, minlength=n_loc)[R_rows]
    R_ptr = np.zeros(R_rows.size + 1, np.int64)
    np.cumsum(R_cnt, out=R_ptr[1:])
    i32 = lambda a: np.ascontiguousarray(a, np.int32)
    return dict(
        lo=lo, hi=hi, n_loc=n_loc,
        L_ptr=i32(L_ptr), L_col=i32(cols[local] - lo), L_val=np.ascontiguousarray(vals[local]),
        H=i32(H), recv_off=i32(recv_off),
        R_rows=i32(R_rows), R_ptr=i32(R_ptr), R_col=i32(np.searchsorted(H, rem_cols)),
        R_val=np.ascontiguousarray(vals[~local]))


def split(A, P: int, r: int) -> dict:
    """Rank r's share of A under the contiguous row-block partition.

    Returns int32/float64 arrays:
      lo, hi                 -- owned global rows [lo, hi)
      L_ptr, L_col, L_val    -- A_L, columns renumbered to local (col - lo)
      H                      -- halo: ascending unique remote global columns
      recv_off               -- [P+1]: H[recv_off[q]:recv_off[q+1]] owned by q
      R_rows, R_ptr, R_col, R_val
                             -- A_R over the rows with remote entries
                                (ascending local row ids), columns = index in H
      send_idx, send_off     -- [P+1]: local indices rank q needs from r,
                                ascending, destinations ascending
    """
    n = A.n_rows
    lo_all = row_blocks(n, P)
    lo, hi = int(lo_all[r]), int(lo_all[r + 1])
    grp = A.row_ptr.astype(np.int64)
    out = _split_rows(grp[lo:hi + 1], A.col_idx, A.val, n, P, r)
    send = []
    send_off = np.zeros(P + 1, np.int64)
    for q in range(P):
        if q != r:
            cq = A.col_idx[grp[lo_all[q]]:grp[lo_all[q + 1]]].astype(np.int64)
            s = np.unique(cq[(cq >= lo) & (cq < hi)]) - lo
        else:
            s = np.zeros(0, np.int64)
        send.append(s)
        send_off[q + 1] = send_off[q] + s.size
    out["send_idx"] = np.ascontiguousarray(np.concatenate(send) if send else np.zeros(0), np.int32)
    out["send_off"] = np.ascontiguousarray(send_off, np.int32)
    return out


def split_local(local, n: int, P: int, r: int, send_idx, send_off) -> dict:
    """The same share from the rank's own rows (global columns) and its send
    lists, as one rank of a distributed code holds it."""
    out = _split_rows(local.row_ptr, local.col_idx, local.val, n, P, r)
    out["send_idx"] = np.ascontiguousarray(send_idx, np.int32)
    out["send_off"] = np.ascontiguousarray(send_off, np.int32)
    return out


def share_reference_local(local, n: int, P: int, r: int, send_idx, send_off, x: np.ndarray,
                          dynamic: bool = False) -> dict:
    """share_reference for a rank-local share: y over the own rows with the
    global x, and the same derived quantities."""
    s = split_local(local, n, P, r, send_idx, send_off)
    y, absax = spmv_dot2(local.row_ptr, local.col_idx, local.val, x, dynamic)
    return _reference_from_parts(s, x, y, absax, dynamic)


def share_reference(A, P: int, r: int, x: np.ndarray, parts: dict | None = None,
                    dynamic: bool = False) -> dict:
    """Everything rank r's share of y = A x produces, from the global A and x.

    y      -- Dot2 over each owned global row (the plain definition)
    yL, yR -- the local product A_L x_L and the remote product A_R x_R (the
              latter scattered onto all owned rows, 0 where a row has no
              remote entry)
    absax  -- |A||x| per owned row, the tolerance scale
    sendbuf -- what the Pack step places in the send buffers: x[lo + send_idx]
    inbox   -- the halo values the other ranks send: x[H]
    """
    s = split(A, P, r) if parts is None else parts
    lo, hi = s["lo"], s["hi"]
    y, absax = spmv_dot2(A.row_ptr[lo:hi + 1], A.col_idx, A.val, x, dynamic)
    return _reference_from_parts(s, x, y, absax, dynamic)


def _reference_from_parts(s, x, y, absax, dynamic) -> dict:
    lo, hi = s["lo"], s["hi"]
    xL = x[lo:hi]
    yL, _ = spmv_dot2(s["L_ptr"], s["L_col"], s["L_val"], xL, dynamic)
    inbox = x[s["H"].astype(np.int64)]
    yRc, _ = spmv_dot2(s["R_ptr"], s["R_col"], s["R_val"], inbox, dynamic)
    yR = np.zeros(hi - lo)
    yR[s["R_rows"].astype(np.int64)] = yRc
    return dict(parts=s, y=y, yL=yL, yR=yR, yR_compressed=yRc, absax=absax,
                sendbuf=xL[s["send_idx"].astype(np.int64)], inbox=inbox)


def within_tolerance(y: np.ndarray, y_ref: np.ndarray, absax: np.ndarray,
                     rel: float = 1e-12) -> np.ndarray:
    """Per-row acceptance: |y - y_ref| <= rel * (|A||x|)_i; a row with
    (|A||x|)_i == 0 must be exactly zero (either sign)."""
    err = np.abs(y - y_ref)
    ok = err <= rel * absax
    zero = absax == 0
    ok[zero] = y[zero] == 0
    return ok


# ---------------------------------------------------------------- exact

def exact_rows(row_ptr, col_idx, val, x):
    """Exact rational value of every row product (tiny inputs only)."""
    out = []
    for i in range(len(row_ptr) - 1):
        s = Fraction(0)
        for k in range(int(row_ptr[i]), int(row_ptr[i + 1])):
            s += Fraction(float(val[k])) * Fraction(float(x[int(col_idx[k])]))
        out.append(s)
    return out


def correctly_rounded(fracs) -> np.ndarray:
    """Round exact rationals once to FP64 (CPython's int/int division rounds
    to nearest)."""
    return np.array([f.numerator / f.denominator for f in fracs], np.float64)


# ---------------------------------------------------------------- plan space
#
# The SpMV program DAG (Sec. III-A, Fig. 3c, whose picture is not in the text).
# Vertex types follow Table II: CPU operations are synchronous; GPU operations
# are asynchronous and must be bound to a stream.  Edges, read from the text:
# start precedes the three independent chains; Pack precedes PostSend, which
# precedes WaitSend; PostRecv precedes WaitRecv, which precedes the remote
# product yR (x_R must be assembled first); yL depends only on start; every
# leaf precedes end.  Unpack runs on yR's stream immediately before yR, so it
# is not a separate choice.

VERTEX_TYPE = {
    "start": "CPU", "Pack": "GPU", "yL": "GPU", "PostSend": "CPU",
    "PostRecv": "CPU", "WaitSend": "CPU", "WaitRecv": "CPU", "yR": "GPU",
    "end": "CPU",
}
DAG_EDGES = [
    ("start", "Pack"), ("start", "yL"), ("start", "PostRecv"),
    ("Pack", "PostSend"), ("PostSend", "WaitSend"),
    ("PostRecv", "WaitRecv"), ("WaitRecv", "yR"),
    ("yL", "end"), ("yR", "end"), ("WaitSend", "end"),
]
GPU_VERTICES = ("Pack", "yL", "yR")


def required_syncs(edges=DAG_EDGES, types=VERTEX_TYPE):
    """Table III applied to every edge u -> v.

    CPU -> anything: nothing.  GPU -> CPU: an event record after u and a
    host synchronisation on it before v, named CER-after-u and CES-b4-v.
    GPU -> GPU on different streams: a record after u and a stream wait before
    v (CER-after-u, CSWE-b4-v); this DAG has no GPU -> GPU edge.  The edges
    into ``end`` need nothing: end is the artificial operation that waits for
    all work (Sec. III-A).
    Returns a list of (u, v, record_name, wait_name).
    """
    out = []
    for u, v in edges:
        if v == "end" or types[u] == "CPU":
            continue
        if types[v] == "CPU":
            out.append((u, v, "CER-after-" + u, "CES-b4-" + v))
    return out


def plan_tokens():
    toks = [v for v in VERTEX_TYPE if v not in ("start", "end")]
    for u, v, rec, wait in required_syncs():
        toks += [rec, wait]
    return toks


def order_is_valid(order) -> bool:
    """Topological w.r.t. the DAG plus sync placement u < record < wait < v."""
    pos = {t: i for i, t in enumerate(order)}
    for u, v in DAG_EDGES:
        if pos[u] >= pos[v]:
            return False
    for u, v, rec, wait in required_syncs():
        if not (pos[u] < pos[rec] < pos[wait] < pos[v]):
            return False
    return True


def canonical_streams(order, assign: dict) -> tuple:
    """Relabel streams by first appearance along the order (Sec. III-C2:
    plans equal up to a bijection of streams are one plan)."""
    relabel = {}
    for t in order:
        if t in assign:
            s = assign[t]
            if s not in relabel:
                relabel[s] = len(relabel)
    return tuple(relabel[assign[g]] for g in GPU_VERTICES)


def plan_space(n_streams: int = 2):
    """All (order, stream map) plans by brute force over permutations.

    ``order`` includes start and end; the stream map gives the canonical
    streams of (Pack, yL, yR)."""
    toks = plan_tokens()
    plans = set()
    for perm in itertools.permutations(toks):
        order = ("start",) + perm + ("end",)
        if not order_is_valid(order):
            continue
        maps = set()
        for ss in itertools.product(range(n_streams), repeat=len(GPU_VERTICES)):
            maps.add(canonical_streams(order, dict(zip(GPU_VERTICES, ss))))
        for m in maps:
            plans.add((order, m))
    return plans


def plan_space_count_formula(n_streams: int = 2) -> int:
    """Closed form: interleavings of the three independent chains times the
    number of stream partitions of the three GPU operations."""
    chains = [5, 3, 1]   # Pack,CER,CES,PostSend,WaitSend | PostRecv,WaitRecv,yR | yL
    inter = math.factorial(sum(chains))
    for c in chains:
        inter //= math.factorial(c)
    # set partitions of 3 labelled items into at most n_streams blocks
    stirling = {1: 1, 2: 3, 3: 1}
    parts = sum(stirling[k] for k in stirling if k <= n_streams)
    return inter * parts
