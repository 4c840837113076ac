"""MI355X (gfx950) row-partitioned SpMV: Python binding of ``libspmv.so``.

Thin ctypes marshalling over the C ABI declared in ``include/spmv.h``; every
step of the SpMV runs in the library's HIP kernels.  Function names match
the C entry points.  Device arrays are passed as torch CUDA tensors (or raw
integer device addresses), host arrays as numpy arrays.

The library must be built first (``python paper_2203_02530_amd/build.py``);
importing this package without it raises ImportError.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libspmv.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build the HIP library with "
        "`python paper_2203_02530_amd/build.py` (no CPU fallback exists)")

# One HIP runtime per process: torch ships its own libamdhip64 (same soname
# as ROCm's), and two runtimes in one process do not share the device.
# Loading torch first makes the library bind to the runtime torch uses.
try:
    import torch  # noqa: F401
except ImportError:  # pure C-ABI use without torch
    torch = None

_lib = ctypes.CDLL(LIB_PATH)


def _hip_runtimes() -> set:
    try:
        with open("/proc/self/maps") as f:
            return {ln.split()[-1] for ln in f if "libamdhip64" in ln}
    except OSError:
        return set()


if len(_hip_runtimes()) > 1:
    raise ImportError("two HIP runtimes are loaded in this process "
                      f"({sorted(_hip_runtimes())}); import torch before any other HIP library")

# ------------------------------------------------------------ constants
SPMV_OK, SPMV_EINVAL, SPMV_ECSR, SPMV_EPLAN = 0, -1, -2, -3
SPMV_ENOMEM, SPMV_EHIP, SPMV_EBUDGET, SPMV_ESTATE = -4, -5, -6, -7

SPMV_OP_START, SPMV_OP_PACK, SPMV_OP_YL, SPMV_OP_POST_SEND = 0, 1, 2, 3
SPMV_OP_POST_RECV, SPMV_OP_WAIT_SEND, SPMV_OP_WAIT_RECV = 4, 5, 6
SPMV_OP_UNPACK, SPMV_OP_YR, SPMV_OP_END, SPMV_N_VERTICES = 7, 8, 9, 10
SPMV_SYNC_CER, SPMV_SYNC_CES, SPMV_SYNC_CSWE = 0x10, 0x20, 0x30
SPMV_MAX_OPS, SPMV_MAX_STREAMS = 24, 8


def SPMV_CER_AFTER(u): return SPMV_SYNC_CER | u
def SPMV_CES_B4(v): return SPMV_SYNC_CES | v
def SPMV_CSWE_B4(v): return SPMV_SYNC_CSWE | v
def SPMV_PEER(op, q): return op | ((q + 1) << 8)


SPMV_F_HOST_ONLY, SPMV_F_PROFILE, SPMV_F_NO_BUFFER = 1, 2, 4
SPMV_F_RESIDENT_SEQUENTIAL = 8
SPMV_KERNEL_VECTOR, SPMV_KERNEL_STREAM = 1, 2

(SPMV_I32_HALO_COLS, SPMV_I32_RECV_OFF, SPMV_I32_SEND_IDX, SPMV_I32_SEND_OFF,
 SPMV_I32_AL_PTR, SPMV_I32_AL_COLS, SPMV_I32_AR_ROWS, SPMV_I32_AR_PTR,
 SPMV_I32_AR_COLS, SPMV_I32_UNPACK_PERM, SPMV_I32_OP_ORDER,
 SPMV_I32_STREAM_MAP, SPMV_I32_TILE_ROW_L, SPMV_I32_TILE_K_L, SPMV_I32_TILE_ROW_R,
 SPMV_I32_TILE_K_R, SPMV_I32_OP_STREAM) = range(17)
(SPMV_F64_AL_VAL, SPMV_F64_AR_VAL, SPMV_F64_SENDBUF, SPMV_F64_RECVBUF,
 SPMV_F64_X_HALO, SPMV_F64_OP_MS, SPMV_F64_OP_COUNT, SPMV_F64_HOST_US,
 SPMV_F64_HOST_COUNT) = range(9)


# ------------------------------------------------------------ structs
class spmv_csr_t(ctypes.Structure):
    _fields_ = [("n_rows", ctypes.c_int32), ("n_cols", ctypes.c_int32),
                ("nnz", ctypes.c_int64), ("row_ptr", ctypes.c_void_p),
                ("col_idx", ctypes.c_void_p), ("val", ctypes.c_void_p)]


class spmv_tune_t(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int32) for k in (
        "kernel_local", "kernel_remote", "lanes_local", "lanes_remote", "rows_local",
        "rows_remote", "chunk_local", "chunk_remote", "width", "xcd_remap", "fuse_unpack",
        "flags", "form")]


class spmv_batch_opts_t(ctypes.Structure):
    _fields_ = [("blocks_per_cu", ctypes.c_int32), ("use_graph", ctypes.c_int32),
                ("xcd_affinity", ctypes.c_int32), ("staging", ctypes.c_int32),
                ("copy_streams", ctypes.c_int32), ("chunks", ctypes.c_int32),
                ("persistent", ctypes.c_int32), ("reserved", ctypes.c_int32 * 1)]


class spmv_batch_info_t(ctypes.Structure):
    _fields_ = [("n_shares", ctypes.c_int32), ("n_blocks", ctypes.c_int32),
                ("n_items", ctypes.c_int64 * 3), ("device_bytes", ctypes.c_int64),
                ("host_link_bytes", ctypes.c_int64), ("chunk", ctypes.c_int32),
                ("width", ctypes.c_int32), ("use_graph", ctypes.c_int32),
                ("xcd_affinity", ctypes.c_int32), ("staging", ctypes.c_int32),
                ("n_chunks", ctypes.c_int32), ("persistent", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["n_items"] = list(self.n_items)
        return d


class spmv_server_opts_t(ctypes.Structure):
    _fields_ = [("budget_bytes", ctypes.c_int64), ("max_inflight", ctypes.c_int32),
                ("max_epochs", ctypes.c_int32), ("max_batch", ctypes.c_int32),
                ("chunk", ctypes.c_int32), ("mode", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 3)]


class spmv_server_stats_t(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("batches", ctypes.c_int64), ("resident_bytes", ctypes.c_int64),
                ("peak_inflight_bytes", ctypes.c_int64), ("arena_bytes", ctypes.c_int64),
                ("peak_inflight", ctypes.c_int32), ("n_matrices", ctypes.c_int32),
                ("mean_batch", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class spmv_mcts_opts_t(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int64), ("seed", ctypes.c_uint64),
                ("c", ctypes.c_double), ("n_streams", ctypes.c_int32),
                ("n_measure", ctypes.c_int32), ("t_measure", ctypes.c_double),
                ("rand", ctypes.c_void_p), ("n_rand", ctypes.c_int64),
                ("reserved", ctypes.c_int64 * 4)]


class spmv_mcts_node_t(ctypes.Structure):
    _fields_ = [("parent", ctypes.c_int32), ("token", ctypes.c_int32),
                ("stream", ctypes.c_int32), ("full", ctypes.c_int32),
                ("n", ctypes.c_int64), ("t_min", ctypes.c_double), ("t_max", ctypes.c_double)]


MCTS_NODE_DTYPE = np.dtype([("parent", np.int32), ("token", np.int32), ("stream", np.int32),
                            ("full", np.int32), ("n", np.int64), ("t_min", np.float64),
                            ("t_max", np.float64)])


class spmv_info_t(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in (
        "n_global", "lo", "n_loc", "nnz_local", "nnz_remote", "n_halo", "n_send",
        "n_remote_rows", "device_bytes")] + [(k, ctypes.c_int32) for k in (
            "nranks", "rank", "n_streams", "n_ops", "kernel_local", "kernel_remote",
            "lanes_local", "lanes_remote", "rows_local", "rows_remote", "chunk_local",
            "chunk_remote", "width", "xcd_remap", "fuse_unpack", "fused_combine",
            "n_tiles_local", "n_tiles_remote", "form_local", "form_remote",
            "n_slices_local", "n_slices_remote", "fine", "device", "resident_grouped")]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


_P = ctypes.c_void_p
_I32, _I64 = ctypes.c_int32, ctypes.c_int64


def _proto(name, args, res=ctypes.c_int):
    f = getattr(_lib, name)
    f.argtypes = args
    f.restype = res
    return f


_proto("spmv_plan_create", [_P, _I32, _I32, _P, _I32, _P, _I32, _P])
_proto("spmv_plan_create_ex", [_P, _I32, _I32, _P, _I32, _P, _I32, _P, _P])
_proto("spmv_plan_create_local", [_P, _I64, _I32, _I32, _P, _P, _P, _I32, _P, _I32, _P, _P])
_proto("spmv_plan_destroy", [_P])
_proto("spmv_exec", [_P, _P, _P, _P])
_proto("spmv_exec_static", [_P, _P, _P, _P])
_proto("spmv_exec_resident", [_P, _P, _P, _P])
_proto("spmv_exec_resident_part", [_P, _I32, _P, _P, _P])
_proto("spmv_plan_device_buffers", [_P, _P, _P, _P, _P])
_proto("spmv_static_scratch_bytes", [], _I64)
_proto("spmv_plan_info", [_P, _P])
_proto("spmv_op_launch", [_P, _I32, _P, _P, _P])
_proto("spmv_plan_reorder", [_P, _P, _I32, _P, _I32])
_proto("spmv_plan_time", [_P, _I32, _P, _P, _P, ctypes.c_double, _I32, _P])
_proto("spmv_plan_get_i32", [_P, _I32, _P, _I64])
_proto("spmv_plan_get_f64", [_P, _I32, _P, _I64])
_proto("spmv_plan_reset_times", [_P])
_proto("spmv_plan_set_profile", [_P, _I32])
_proto("spmv_plan_inbox", [_P, _P, _P])
_proto("spmv_plan_outbox", [_P, _P, _P])
_proto("spmv_plan_validate", [_I32, _P, _I32, _P, _I32])
_proto("spmv_plan_space_count", [_I32, _I32, _P])
_proto("spmv_plan_space_get", [_I32, _I32, _I64, _P, _P, _P])
_proto("spmv_op_name", [_I32, ctypes.c_char_p, _I32])
_proto("spmv_mcts_run_table", [_I32, _P, _I64, _P, _P, _P, _I64, _P, _P, _I64, _P])
_proto("spmv_mcts_run", [_P, _I32, _P, _P, _P, _P, _P, _P, _I64, _P, _P, _I64, _P])
COST_FN = ctypes.CFUNCTYPE(ctypes.c_double, ctypes.POINTER(ctypes.c_int32),
                           ctypes.POINTER(ctypes.c_int32), ctypes.c_int32, ctypes.c_void_p)
_proto("spmv_mcts_run_seq", [_P, _I32, _P, _P, _P, _I32, COST_FN, _P, _P, _P, _P, _I32, _P,
                             _I64, _P, _P, _I64, _P])
_proto("spmv_fine_tokens", [_P, _P, _I32, _P])
_proto("spmv_fine_default", [_P, _P, _P, _I32, _P])
_proto("spmv_fine_count", [_P, _I32, _P])
_proto("spmv_plan_set_fine", [_P, _P, _P, _I32, _I32])
_proto("spmv_fine_validate", [_P, _P, _P, _I32, _I32])
_proto("spmv_hbm_probe", [_I32, _P, _P, _I64, _I32, _P])
_proto("spmv_gathers_per_probe_block", [], _I64)
_proto("spmv_batch_create", [_P, _I32, _P, _P])
_proto("spmv_batch_exec", [_P, _P, _P, _P])
_proto("spmv_batch_info", [_P, _P])
_proto("spmv_batch_destroy", [_P])
_proto("spmv_server_create", [_P, _P])
_proto("spmv_server_add_matrix", [_P, _P, _P])
_proto("spmv_server_start", [_P])
_proto("spmv_server_submit", [_P, _I32, _P, _P, _I64])
_proto("spmv_server_poll", [_P, _P, _P, _I32, _P])
_proto("spmv_server_drain", [_P])
_proto("spmv_server_run_trace", [_P, _I64, _P, _P, _P, _P, _P, _P])
_proto("spmv_server_stats", [_P, _P])
_proto("spmv_server_destroy", [_P])
_proto("spmv_last_error", [], ctypes.c_char_p)
_proto("spmv_version", [], ctypes.c_char_p)


class SpmvError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[{code}] {msg}")
        self.code = code


def _check(rc: int) -> int:
    if rc < 0:
        raise SpmvError(rc, _lib.spmv_last_error().decode(errors="replace"))
    return rc


def _addr(a) -> int:
    """Address of a torch tensor, numpy array, int or None."""
    if a is None:
        return 0
    if isinstance(a, int):
        return a
    if isinstance(a, np.ndarray):
        return a.ctypes.data
    return int(a.data_ptr())


# Per plan: (n_loc, device), cached at the first check and dropped when the
# plan is destroyed (a later plan may reuse the handle's address).
_PLAN_META: dict = {}
# Per batch: the (n_loc, device) of each share, recorded at creation.
_BATCH_META: dict = {}


def _plan_meta(plan):
    m = _PLAN_META.get(plan)
    if m is None:
        info = spmv_plan_info(plan)
        m = (int(info["n_loc"]), int(info["device"]))
        _PLAN_META[plan] = m
    return m


def _dev_vec(a, n: int, device: int, name: str) -> int:
    """Address of a device vector of at least n FP64 entries, checked: a
    contiguous float64 torch CUDA tensor on `device`, or None when n == 0.
    A plain int is taken as a raw device address the caller vouches for
    (the library cannot inspect it).  Anything else -- a host array, a CPU
    tensor, another dtype, a strided view, too few entries, another device
    -- raises before any launch."""
    if a is None:
        if n > 0:
            raise ValueError(f"{name} is None but the plan has {n} rows")
        return 0
    if isinstance(a, int):
        return a
    if isinstance(a, np.ndarray):
        raise TypeError(f"{name} is a host numpy array; pass a device tensor")
    if torch is None or not isinstance(a, torch.Tensor):
        raise TypeError(f"{name} must be a torch CUDA tensor, got {type(a).__name__}")
    if not a.is_cuda:
        raise ValueError(f"{name} is on {a.device}, not on a GPU")
    if a.dtype != torch.float64:
        raise TypeError(f"{name} has dtype {a.dtype}; the library computes in float64")
    if not a.is_contiguous():
        raise ValueError(f"{name} is not contiguous")
    if a.numel() < n:
        raise ValueError(f"{name} has {a.numel()} entries, the plan needs {n}")
    if device >= 0 and a.device.index != device:
        raise ValueError(f"{name} is on cuda:{a.device.index}, the plan on cuda:{device}")
    return int(a.data_ptr())


def _plan_vecs(plan, x, y, need_x: bool = True, need_y: bool = True):
    n, dev = _plan_meta(plan)
    return (_dev_vec(x, n if need_x else 0, dev, "x") if (need_x or x is not None) else 0,
            _dev_vec(y, n if need_y else 0, dev, "y") if (need_y or y is not None) else 0)


def _stream_handle(stream) -> int:
    if stream is None:
        return 0
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)


def _i32(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.int32)


def make_csr(A):
    """spmv_csr_t view of a CSR (anything with n_rows, n_cols, row_ptr,
    col_idx, val).  Returns (struct, keepalive)."""
    rp = _i32(A.row_ptr)
    ci = _i32(A.col_idx)
    va = np.ascontiguousarray(A.val, dtype=np.float64)
    c = spmv_csr_t(int(A.n_rows), int(A.n_cols), int(rp[-1]) if rp.size else 0,
                   rp.ctypes.data, ci.ctypes.data, va.ctypes.data)
    return c, (rp, ci, va)


# ------------------------------------------------------------ entry points
def spmv_plan_create(A, nranks: int, rank: int, op_order=None, stream_map=None,
                     n_streams: int = 2, tune: spmv_tune_t | dict | None = None):
    """Build a plan for rank ``rank`` of ``nranks``; returns the plan handle."""
    c, keep = make_csr(A)
    ops = None if op_order is None else _i32(op_order)
    smap = _smap_array(stream_map)
    if isinstance(tune, dict):
        t = spmv_tune_t()
        for k, v in tune.items():
            setattr(t, k, v)
        tune = t
    out = ctypes.c_void_p()
    _check(_lib.spmv_plan_create_ex(
        ctypes.byref(c), nranks, rank, _addr(ops), 0 if ops is None else ops.size,
        _addr(smap), n_streams, ctypes.byref(tune) if tune is not None else None,
        ctypes.byref(out)))
    del keep
    return out.value


def spmv_plan_create_local(local, n_global: int, nranks: int, rank: int, send_idx, send_off,
                           op_order=None, stream_map=None, n_streams: int = 2, tune=None):
    """Plan from the rank's own rows (global columns) and its send lists."""
    c, keep = make_csr(local)
    si = _i32(send_idx)
    so = _i32(send_off)
    ops = None if op_order is None else _i32(op_order)
    smap = _smap_array(stream_map)
    if isinstance(tune, dict):
        t = spmv_tune_t()
        for k, v in tune.items():
            setattr(t, k, v)
        tune = t
    out = ctypes.c_void_p()
    _check(_lib.spmv_plan_create_local(
        ctypes.byref(c), n_global, nranks, rank, _addr(si) if si.size else None, _addr(so),
        _addr(ops), 0 if ops is None else ops.size, _addr(smap), n_streams,
        ctypes.byref(tune) if tune is not None else None, ctypes.byref(out)))
    del keep
    return out.value


def spmv_plan_destroy(plan) -> None:
    _PLAN_META.pop(plan, None)
    _check(_lib.spmv_plan_destroy(plan))


def spmv_exec(plan, x, y, stream=None) -> None:
    """y = (A x) over the plan's rows; x, y contiguous float64 CUDA tensors
    of at least n_loc entries on the plan's device (checked)."""
    xa, ya = _plan_vecs(plan, x, y)
    _check(_lib.spmv_exec(plan, xa, ya, _stream_handle(stream)))


def spmv_exec_static(plan, x, y, stream=None) -> None:
    """spmv_exec with the exec's intermediate data in the library's fixed
    per-device scratch array (allocates nothing); same checks and results."""
    xa, ya = _plan_vecs(plan, x, y)
    _check(_lib.spmv_exec_static(plan, xa, ya, _stream_handle(stream)))


def spmv_exec_resident(plan, x, y, stream=None) -> None:
    """The share's device work (Pack, y_L, Unpack, y_R) on ``stream`` with
    the halo already in the plan's device receive buffer; asynchronous."""
    xa, ya = _plan_vecs(plan, x, y)
    _check(_lib.spmv_exec_resident(plan, xa, ya, _stream_handle(stream)))


def spmv_exec_resident_part(plan, part: int, x, y, stream=None) -> None:
    """One of the two grouped launches of the resident step (0: Pack, y_L
    and the column-slab tiles; 1: the slab sums into y); asynchronous."""
    xa, ya = _plan_vecs(plan, x, y)
    _check(_lib.spmv_exec_resident_part(plan, int(part), xa, ya, _stream_handle(stream)))


def spmv_plan_device_buffers(plan) -> dict:
    """Device addresses and lengths of the plan's send and receive buffers."""
    sd, rd = ctypes.c_void_p(), ctypes.c_void_p()
    ns, nh = ctypes.c_int64(), ctypes.c_int64()
    _check(_lib.spmv_plan_device_buffers(plan, ctypes.byref(sd), ctypes.byref(ns),
                                         ctypes.byref(rd), ctypes.byref(nh)))
    return {"send": sd.value or 0, "n_send": ns.value, "recv": rd.value or 0,
            "n_halo": nh.value}


def spmv_static_scratch_bytes() -> int:
    return int(_lib.spmv_static_scratch_bytes())


def spmv_op_launch(plan, op: int, x=None, y=None, stream=None) -> None:
    """Launch one GPU op of the plan asynchronously on ``stream``; x is
    checked for Pack and y_L, y for y_L and y_R."""
    xa, ya = _plan_vecs(plan, x, y, need_x=op in (SPMV_OP_PACK, SPMV_OP_YL),
                        need_y=op in (SPMV_OP_YL, SPMV_OP_YR))
    _check(_lib.spmv_op_launch(plan, op, xa, ya, _stream_handle(stream)))


def _smap_array(stream_map):
    if stream_map is None:
        return None
    smap = np.full(SPMV_N_VERTICES, -1, np.int32)
    if isinstance(stream_map, dict):
        for k, v in stream_map.items():
            smap[k] = v
    else:
        smap[:len(stream_map)] = stream_map
    return smap


def spmv_plan_reorder(plan, op_order, stream_map=None, n_streams: int = 2) -> None:
    """Swap the plan's operation order and stream map (same share)."""
    ops = _i32(op_order)
    smap = _smap_array(stream_map)
    _check(_lib.spmv_plan_reorder(plan, _addr(ops), ops.size, _addr(smap), n_streams))


def spmv_plan_time(plans, xs, ys, stream=None, t_measure: float = 0.01,
                   n_measure: int = 5) -> np.ndarray:
    """The paper's protocol: per measurement, repeat exec for t_measure
    seconds, rotating over `plans` (a plan handle or a list of replicas) and
    their x / y; returns seconds per exec for each measurement."""
    if not isinstance(plans, (list, tuple)):
        plans, xs, ys = [plans], [xs], [ys]
    n = len(plans)
    pa = (ctypes.c_void_p * n)(*plans)
    xa, ya = _vec_tables(plans, xs, ys)
    out = np.empty(n_measure, np.float64)
    _check(_lib.spmv_plan_time(pa, n, xa, ya, _stream_handle(stream), t_measure, n_measure,
                               out.ctypes.data))
    return out


def _vec_tables(plans, xs, ys):
    """ctypes tables of the checked x / y addresses of each plan."""
    if len(xs) != len(plans) or len(ys) != len(plans):
        raise ValueError("need one x and one y per plan")
    n = len(plans)
    pairs = [_plan_vecs(p, x, y) for p, x, y in zip(plans, xs, ys)]
    return ((ctypes.c_void_p * n)(*[a or None for a, _ in pairs]),
            (ctypes.c_void_p * n)(*[b or None for _, b in pairs]))


def spmv_plan_info(plan) -> dict:
    info = spmv_info_t()
    _check(_lib.spmv_plan_info(plan, ctypes.byref(info)))
    return info.as_dict()


def _tiles_r(i):
    # form 5 keeps the 8 column slabs' tiles one after another, each with
    # its closing entry
    if i["form_remote"] == 5:
        return i["n_tiles_remote"] + SLABS
    return i["n_tiles_remote"] + 1 if i["form_remote"] in (1, 4) else 0


SLABS = 8   # column slabs of form 5, one per XCD


_I32_LEN = {
    SPMV_I32_HALO_COLS: lambda i: i["n_halo"], SPMV_I32_RECV_OFF: lambda i: i["nranks"] + 1,
    SPMV_I32_SEND_IDX: lambda i: i["n_send"], SPMV_I32_SEND_OFF: lambda i: i["nranks"] + 1,
    SPMV_I32_AL_PTR: lambda i: i["n_loc"] + 1, SPMV_I32_AL_COLS: lambda i: i["nnz_local"],
    SPMV_I32_AR_ROWS: lambda i: i["n_remote_rows"],
    SPMV_I32_AR_PTR: lambda i: i["n_remote_rows"] + 1,
    SPMV_I32_AR_COLS: lambda i: i["nnz_remote"], SPMV_I32_UNPACK_PERM: lambda i: i["n_halo"],
    SPMV_I32_OP_ORDER: lambda i: i["n_ops"], SPMV_I32_STREAM_MAP: lambda i: SPMV_N_VERTICES,
    SPMV_I32_OP_STREAM: lambda i: i["n_ops"],
    SPMV_I32_TILE_ROW_L: lambda i: i["n_tiles_local"] + 1 if i["form_local"] in (1, 4) else 0,
    SPMV_I32_TILE_K_L: lambda i: i["n_tiles_local"] + 1 if i["form_local"] in (1, 4) else 0,
    SPMV_I32_TILE_ROW_R: lambda i: _tiles_r(i),
    SPMV_I32_TILE_K_R: lambda i: _tiles_r(i),
}
_F64_LEN = {
    SPMV_F64_AL_VAL: lambda i: i["nnz_local"], SPMV_F64_AR_VAL: lambda i: i["nnz_remote"],
    SPMV_F64_SENDBUF: lambda i: i["n_send"], SPMV_F64_RECVBUF: lambda i: i["n_halo"],
    SPMV_F64_X_HALO: lambda i: i["n_halo"], SPMV_F64_OP_MS: lambda i: SPMV_N_VERTICES + 1,
    SPMV_F64_OP_COUNT: lambda i: SPMV_N_VERTICES + 1,
    SPMV_F64_HOST_US: lambda i: i["n_ops"], SPMV_F64_HOST_COUNT: lambda i: 1,
}


def spmv_plan_get_i32(plan, which: int) -> np.ndarray:
    n = _I32_LEN[which](spmv_plan_info(plan))
    out = np.empty(max(n, 1), np.int32)
    _check(_lib.spmv_plan_get_i32(plan, which, out.ctypes.data, out.size))
    return out[:n]


def spmv_plan_get_f64(plan, which: int) -> np.ndarray:
    n = _F64_LEN[which](spmv_plan_info(plan))
    out = np.empty(max(n, 1), np.float64)
    _check(_lib.spmv_plan_get_f64(plan, which, out.ctypes.data, out.size))
    return out[:n]


def spmv_plan_set_profile(plan, on: bool = True, host: bool = False) -> None:
    """Per-op GPU event timing (``on``) and the host timeline (``host``)."""
    _check(_lib.spmv_plan_set_profile(plan, (1 if on else 0) | (2 if host else 0)))


def spmv_plan_reset_times(plan) -> None:
    _check(_lib.spmv_plan_reset_times(plan))


def _mailbox(fn, plan) -> np.ndarray:
    p = ctypes.c_void_p()
    n = ctypes.c_int64()
    _check(fn(plan, ctypes.byref(p), ctypes.byref(n)))
    if n.value == 0:
        return np.zeros(0, np.float64)
    buf = (ctypes.c_double * n.value).from_address(p.value)
    return np.frombuffer(buf, dtype=np.float64)


def spmv_plan_inbox(plan) -> np.ndarray:
    """Writable numpy view of the plan's pinned inbox (halo order)."""
    return _mailbox(_lib.spmv_plan_inbox, plan)


def spmv_plan_outbox(plan) -> np.ndarray:
    """Numpy view of the plan's pinned outbox (packed send buffer)."""
    return _mailbox(_lib.spmv_plan_outbox, plan)


def spmv_plan_validate(nranks: int, op_order, stream_map=None, n_streams: int = 2) -> int:
    """Returns SPMV_OK or the negative error code (no exception)."""
    ops = _i32(op_order)
    smap = None if stream_map is None else _i32(stream_map)
    return _lib.spmv_plan_validate(nranks, _addr(ops), ops.size, _addr(smap), n_streams)


def spmv_plan_space_count(nranks: int, n_streams: int) -> int:
    n = ctypes.c_int64()
    _check(_lib.spmv_plan_space_count(nranks, n_streams, ctypes.byref(n)))
    return n.value


def spmv_plan_space_get(nranks: int, n_streams: int, index: int):
    """(op_order int32 array, stream_map int32 array[SPMV_N_VERTICES])."""
    ops = np.empty(SPMV_MAX_OPS, np.int32)
    smap = np.empty(SPMV_N_VERTICES, np.int32)
    n = ctypes.c_int32()
    _check(_lib.spmv_plan_space_get(nranks, n_streams, index, ops.ctypes.data,
                                    ctypes.byref(n), smap.ctypes.data))
    return ops[:n.value].copy(), smap


def _mcts_opts(iterations, seed, c, n_streams, n_measure, t_measure, rand):
    o = spmv_mcts_opts_t()
    o.iterations, o.seed, o.c = int(iterations), int(seed), float(c)
    o.n_streams, o.n_measure, o.t_measure = int(n_streams), int(n_measure), float(t_measure)
    keep = None
    if rand is not None:
        keep = np.ascontiguousarray(rand, dtype=np.uint64)
        o.rand, o.n_rand = keep.ctypes.data, keep.size
    return o, keep


def _mcts_result(fn, args, o, cap):
    idx = np.empty(cap, np.int64)
    tim = np.empty(cap, np.float64)
    n = ctypes.c_int64()
    n_nodes = ctypes.c_int64()
    node_cap = cap * SPMV_MAX_OPS + 1     # a rollout creates at most one node per token
    nodes = np.zeros(node_cap, MCTS_NODE_DTYPE)
    _check(fn(*args, ctypes.byref(o), idx.ctypes.data, tim.ctypes.data, cap, ctypes.byref(n),
              nodes.ctypes.data, node_cap, ctypes.byref(n_nodes)))
    k = min(n.value, cap)
    return {"index": idx[:k].copy(), "time": tim[:k].copy(),
            "nodes": nodes[:min(n_nodes.value, node_cap)].copy()}


def spmv_mcts_run_table(nranks: int, cost, iterations: int = 0, seed: int = 0, c: float = 0.0,
                        n_streams: int = 2, rand=None) -> dict:
    """Tree search over the plan space with cost[i] as plan i's time.
    Returns {index, time (per rollout, in order), nodes (structured array of
    the final tree, MCTS_NODE_DTYPE)}."""
    cost = np.ascontiguousarray(cost, dtype=np.float64)
    o, keep = _mcts_opts(iterations, seed, c, n_streams, 1, 0.01, rand)
    cap = int(iterations) if iterations > 0 else cost.size
    return _mcts_result(_lib.spmv_mcts_run_table, (nranks, cost.ctypes.data, cost.size), o, cap)


def spmv_mcts_run(plans, xs, ys, stream=None, iterations: int = 0, seed: int = 0,
                  c: float = 0.0, n_streams: int = 2, t_measure: float = 0.01,
                  n_measure: int = 1, rand=None) -> dict:
    """Tree search timing every rollout on the device (the plans, a handle
    or a list of replicas, are re-ordered in place).  Same result as
    spmv_mcts_run_table."""
    if not isinstance(plans, (list, tuple)):
        plans, xs, ys = [plans], [xs], [ys]
    n = len(plans)
    pa = (ctypes.c_void_p * n)(*plans)
    xa, ya = _vec_tables(plans, xs, ys)
    o, keep = _mcts_opts(iterations, seed, c, n_streams, n_measure, t_measure, rand)
    nranks = spmv_plan_info(plans[0])["nranks"]
    cap = int(iterations) if iterations > 0 else spmv_plan_space_count(nranks, max(n_streams, 1))
    return _mcts_result(_lib.spmv_mcts_run, (pa, n, xa, ya, _stream_handle(stream)), o, cap)


def spmv_mcts_run_seq(plans, xs=None, ys=None, stream=None, fine: bool = False, cost=None,
                      iterations: int = 0, seed: int = 0, c: float = 0.0, n_streams: int = 2,
                      t_measure: float = 0.01, n_measure: int = 1, rand=None,
                      max_rollouts: int = 100000) -> dict:
    """Tree search over the coarse or the fine-grained DAG of the plans'
    share.  ``cost(ops, streams)`` (numpy int32 arrays) gives a rollout's
    time on the host; without it rollouts are timed on the device.  Returns
    {ops [k, n_ops], streams [k, n_ops], time [k], nodes}."""
    if not isinstance(plans, (list, tuple)):
        plans = [plans]
        xs = [xs] if xs is not None else None
        ys = [ys] if ys is not None else None
    n = len(plans)
    pa = (ctypes.c_void_p * n)(*plans)
    xa, ya = _vec_tables(plans, xs, ys) if xs and ys else (None, None)
    o, keep = _mcts_opts(iterations, seed, c, n_streams, n_measure, t_measure, rand)
    if fine:
        max_ops = len(spmv_fine_tokens(plans[0]))
    else:
        max_ops = SPMV_MAX_OPS
    cap = int(iterations) if iterations > 0 else int(max_rollouts)
    ops = np.full((cap, max_ops), -1, np.int32)
    sts = np.full((cap, max_ops), -1, np.int32)
    tim = np.empty(cap, np.float64)
    nn = ctypes.c_int64()
    n_nodes = ctypes.c_int64()
    node_cap = cap * max_ops + 1
    nodes = np.zeros(node_cap, MCTS_NODE_DTYPE)
    err = []

    def _cb(po, ps, k, _user):
        try:
            a = np.ctypeslib.as_array(po, shape=(k,)).copy()
            b = np.ctypeslib.as_array(ps, shape=(k,)).copy()
            return float(cost(a, b))
        except Exception as e:          # reported after the call returns
            err.append(e)
            return 0.0
    cb = COST_FN(_cb) if cost is not None else COST_FN()
    _check(_lib.spmv_mcts_run_seq(pa, n, xa, ya, _stream_handle(stream), 1 if fine else 0, cb,
                                  None, ctypes.byref(o), ops.ctypes.data, sts.ctypes.data,
                                  max_ops, tim.ctypes.data, cap, ctypes.byref(nn),
                                  nodes.ctypes.data, node_cap, ctypes.byref(n_nodes)))
    if err:
        raise err[0]
    k = min(nn.value, cap)
    n_ops = int(np.max(np.sum(ops[:k] >= 0, axis=1))) if k else 0
    return {"ops": ops[:k, :n_ops].copy(), "streams": sts[:k, :n_ops].copy(),
            "time": tim[:k].copy(), "nodes": nodes[:min(n_nodes.value, node_cap)].copy()}


def spmv_fine_tokens(plan) -> np.ndarray:
    n = ctypes.c_int32()
    _check(_lib.spmv_fine_tokens(plan, None, 0, ctypes.byref(n)))
    out = np.empty(n.value, np.int32)
    _check(_lib.spmv_fine_tokens(plan, out.ctypes.data, n.value, ctypes.byref(n)))
    return out


def spmv_fine_default(plan):
    """(ops, streams) of the default fine-grained order."""
    cap = len(spmv_fine_tokens(plan))
    ops = np.empty(cap, np.int32)
    sts = np.empty(cap, np.int32)
    n = ctypes.c_int32()
    _check(_lib.spmv_fine_default(plan, ops.ctypes.data, sts.ctypes.data, cap, ctypes.byref(n)))
    return ops[:n.value].copy(), sts[:n.value].copy()


def spmv_fine_count(plan, n_streams: int = 2) -> float:
    c = ctypes.c_double()
    _check(_lib.spmv_fine_count(plan, n_streams, ctypes.byref(c)))
    return c.value


def spmv_plan_set_fine(plan, op_order=None, op_stream=None, n_streams: int = 2) -> None:
    if op_order is None:
        _check(_lib.spmv_plan_set_fine(plan, None, None, 0, n_streams))
        return
    ops = _i32(op_order)
    sts = _i32(op_stream if op_stream is not None else np.zeros(ops.size, np.int32))
    _check(_lib.spmv_plan_set_fine(plan, ops.ctypes.data, sts.ctypes.data, ops.size, n_streams))


def spmv_fine_validate(plan, op_order, op_stream=None, n_streams: int = 2) -> int:
    ops = _i32(op_order)
    sts = _i32(op_stream if op_stream is not None else np.zeros(ops.size, np.int32))
    return _check(_lib.spmv_fine_validate(plan, ops.ctypes.data, sts.ctypes.data, ops.size,
                                          n_streams))


def spmv_op_name(op: int) -> str:
    buf = ctypes.create_string_buffer(64)
    _check(_lib.spmv_op_name(op, buf, 64))
    return buf.value.decode()


def spmv_gathers_per_probe_block() -> int:
    return int(_lib.spmv_gathers_per_probe_block())


def spmv_hbm_probe(mode: int, src, dst, nbytes: int, blocks: int = 0, stream=None) -> None:
    """Launch the read (mode 0), copy (mode 1) or gather (modes 2, 3) probe.
    src and dst are contiguous CUDA tensors: src holds at least nbytes, dst
    at least nbytes (copy) or one double per block (the others)."""
    grid = blocks or 2048
    for name, t, need in (("src", src, nbytes), ("dst", dst, nbytes if mode == 1 else 8 * grid)):
        if not (hasattr(t, "is_cuda") and t.is_cuda and t.is_contiguous()):
            raise TypeError(f"{name} must be a contiguous CUDA tensor")
        if t.numel() * t.element_size() < need:
            raise ValueError(f"{name} holds {t.numel() * t.element_size()} bytes, needs {need}")
    _check(_lib.spmv_hbm_probe(mode, _addr(src), _addr(dst), nbytes, blocks,
                               _stream_handle(stream)))


def spmv_batch_create(plans, opts: dict | None = None):
    """Batch over a list of plan handles; returns the batch handle."""
    arr = (ctypes.c_void_p * len(plans))(*plans)
    o = spmv_batch_opts_t()
    for k, v in (opts or {}).items():
        setattr(o, k, v)
    out = ctypes.c_void_p()
    _check(_lib.spmv_batch_create(arr, len(plans), ctypes.byref(o), ctypes.byref(out)))
    _BATCH_META[out.value] = [_plan_meta(p) for p in plans]
    return out.value


def spmv_batch_exec(batch, xs, ys, stream=None) -> None:
    """xs, ys: sequences of device tensors, one per share, each checked
    like spmv_exec's against its share."""
    meta = _BATCH_META.get(batch)
    if meta is None:
        raise ValueError("unknown batch handle")
    if len(xs) != len(meta) or len(ys) != len(meta):
        raise ValueError(f"the batch has {len(meta)} shares; got {len(xs)} x and {len(ys)} y")
    n = len(xs)
    xa = (ctypes.c_void_p * n)(*[_dev_vec(v, m[0], m[1], f"x[{i}]") or None
                                 for i, (v, m) in enumerate(zip(xs, meta))])
    ya = (ctypes.c_void_p * n)(*[_dev_vec(v, m[0], m[1], f"y[{i}]") or None
                                 for i, (v, m) in enumerate(zip(ys, meta))])
    _check(_lib.spmv_batch_exec(batch, xa, ya, _stream_handle(stream)))


def spmv_batch_info(batch) -> dict:
    info = spmv_batch_info_t()
    _check(_lib.spmv_batch_info(batch, ctypes.byref(info)))
    return info.as_dict()


def spmv_batch_destroy(batch) -> None:
    _BATCH_META.pop(batch, None)
    _check(_lib.spmv_batch_destroy(batch))


def spmv_server_create(opts: dict | None = None):
    o = spmv_server_opts_t()
    for k, v in (opts or {}).items():
        setattr(o, k, v)
    out = ctypes.c_void_p()
    _check(_lib.spmv_server_create(ctypes.byref(o), ctypes.byref(out)))
    return out.value


def spmv_server_add_matrix(srv, A) -> int:
    c, keep = make_csr(A)
    mid = ctypes.c_int32()
    _check(_lib.spmv_server_add_matrix(srv, ctypes.byref(c), ctypes.byref(mid)))
    del keep
    return mid.value


def spmv_server_start(srv) -> None:
    _check(_lib.spmv_server_start(srv))


def spmv_server_submit(srv, matrix: int, x_host, y_host, tag: int) -> None:
    """x_host / y_host: pinned host arrays (torch pinned tensors or addresses)."""
    _check(_lib.spmv_server_submit(srv, matrix, _addr(x_host), _addr(y_host), tag))


def spmv_server_poll(srv, cap: int = 4096):
    tags = np.empty(cap, np.int64)
    lat = np.empty(cap, np.float64)
    n = ctypes.c_int32()
    _check(_lib.spmv_server_poll(srv, tags.ctypes.data, lat.ctypes.data, cap, ctypes.byref(n)))
    return tags[:n.value].copy(), lat[:n.value].copy()


def spmv_server_drain(srv) -> None:
    _check(_lib.spmv_server_drain(srv))


def spmv_server_run_trace(srv, matrix, arrival_s, xs, ys):
    """Replay an arrival trace natively; returns (latency seconds per request,
    wall seconds from first arrival to last completion)."""
    n = len(matrix)
    m = np.ascontiguousarray(matrix, np.int32)
    a = np.ascontiguousarray(arrival_s, np.float64)
    xa = (ctypes.c_void_p * n)(*[_addr(v) for v in xs])
    ya = (ctypes.c_void_p * n)(*[_addr(v) for v in ys])
    lat = np.empty(n, np.float64)
    wall = ctypes.c_double()
    _check(_lib.spmv_server_run_trace(srv, n, m.ctypes.data, a.ctypes.data, xa, ya,
                                      lat.ctypes.data, ctypes.byref(wall)))
    return lat, wall.value


def spmv_server_stats(srv) -> dict:
    st = spmv_server_stats_t()
    _check(_lib.spmv_server_stats(srv, ctypes.byref(st)))
    return st.as_dict()


def spmv_server_destroy(srv) -> None:
    _check(_lib.spmv_server_destroy(srv))


def spmv_last_error() -> str:
    return _lib.spmv_last_error().decode(errors="replace")


def spmv_version() -> str:
    return _lib.spmv_version().decode()
