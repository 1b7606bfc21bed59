"""idsketch: CountSketch / TensorSketch interpolative decomposition on MI355X.

Thin Python binding over the C-ABI library ``libidsketch.so`` (declared in
``include/idsketch.h``).  It only marshals arguments: torch tensors provide
device memory and the current HIP stream, and every step of the computation
runs in the library's HIP kernels.  There is no fallback: if the library is
missing or no GPU is present, calls raise.

Method (Malik & Becker, "Fast randomized matrix and tensor interpolative
decomposition using CountSketch"):
  * :func:`id_sketch`  -- Algorithm 2, CountSketch Y1 = S A (Section 1.3), with
    an optional Gaussian projection Y = G Y1 (Section 1.2.1).
  * :func:`id_select`  -- Algorithm 1 on a sketch: rank-k column-pivoted QR,
    J and P = [I, R11^{-1} R12] Pi^T.
  * :func:`matrix_id`  -- the two above in sequence.
  * :func:`tensor_id`  -- Algorithm 3: TensorSketch, Algorithm 1,
    lambda_hat_k = lambda_{j_k} sum_r p_kr.
"""
from __future__ import annotations

import atexit
import ctypes
import os

__all__ = ["lib", "lib_path", "BatchedPlan", "batched_plan", "id_batched", "BatchedGraph", "batched_graph", "profile_enable", "profile_stages",
           "profile_read", "profile_reset", "id_sketch", "id_project", "id_select", "id_select_noalloc",
           "matrix_id", "tensor_id", "tensor_id_csc", "gaussian_sketch", "gaussian_id", "check_status", "set_wait_limit", "select_plan_info", "stream_read", "tune_set", "tune_get",
           "finalize", "IdsError", "F64", "F32", "BF16", "HASH_FULLRANK", "CHECK_FINITE", "EXPORTED",
           "OK", "ETIMEOUT", "ERANKDEF", "ENONFINITE"]

_HERE = os.path.dirname(os.path.abspath(__file__))
lib_path = os.path.join(_HERE, "libidsketch.so")

F64, F32, BF16 = 0, 1, 2
DENSE, CSR = 0, 1
HASH_FULLRANK = 1
CHECK_FINITE = 2
DETERMINISTIC = 4
# status codes (returned by calls: 0..4; written to device status words: 0, 5..7)
OK, EINVAL, EDTYPE, EWORKSPACE, EHIP, ETIMEOUT, ERANKDEF, ENONFINITE = range(8)

EXPORTED = ["ids_sketch_workspace_size", "id_sketch", "id_project", "ids_gaussian_workspace_size",
            "id_gaussian_sketch", "ids_select_workspace_size",
            "id_select", "id_select_noalloc", "ids_set_wait_limit", "ids_select_plan_info", "ids_stream_read", "ids_tune_set", "ids_tune_get", "ids_tensor_workspace_size", "tensor_id", "ids_tensor_csc_workspace_size", "tensor_id_csc",
            "ids_batched_plan_size", "ids_batched_plan", "id_batched", "ids_batched_graph_create",
            "ids_batched_graph_launch", "ids_batched_graph_destroy", "ids_profile_enable", "ids_profile_stages",
            "ids_profile_read", "ids_profile_reset", "ids_finalize", "ids_status_string", "ids_last_error"]

c_i64 = ctypes.c_int64
c_i32 = ctypes.c_int32
c_u64 = ctypes.c_uint64
c_u32 = ctypes.c_uint32
c_vp = ctypes.c_void_p
c_sz = ctypes.c_size_t


class IdsMatrix(ctypes.Structure):
    _fields_ = [("fmt", c_i32), ("dtype", c_i32), ("m", c_i64), ("n", c_i64), ("ld", c_i64),
                ("nnz", c_i64), ("val", c_vp), ("rowptr", c_vp), ("colind", c_vp)]


class IdsSketchCfg(ctypes.Structure):
    _fields_ = [("l1", c_i64), ("l", c_i64), ("seed", c_u64), ("tag", c_u64), ("flags", c_u32),
                ("acc", c_i32), ("proj", c_i32), ("G", c_vp), ("fr_pi", c_vp), ("fr_x", c_vp), ("status", c_vp)]


class IdsError(RuntimeError):
    pass


_lib = None


def lib():
    """Load libidsketch.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(lib_path):
            raise ImportError(f"{lib_path} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'`")
        L = ctypes.CDLL(lib_path)
        P = ctypes.POINTER
        L.ids_sketch_workspace_size.argtypes = [P(IdsMatrix), P(IdsSketchCfg), P(c_sz)]
        L.id_sketch.argtypes = [P(IdsMatrix), P(IdsSketchCfg), c_vp, c_i32, c_i64, c_vp, c_sz, c_vp]
        L.id_project.argtypes = [c_i32, c_i64, c_i64, c_i64, c_vp, c_vp, c_i64, c_vp, c_i64, c_vp]
        L.ids_gaussian_workspace_size.argtypes = [P(IdsMatrix), c_i64, P(c_sz)]
        L.id_gaussian_sketch.argtypes = [P(IdsMatrix), c_i64, c_vp, c_vp, c_i64, c_vp, c_sz, c_vp]
        L.ids_select_workspace_size.argtypes = [c_i64, c_i64, c_i64, P(c_sz)]
        L.id_select.argtypes = [c_vp, c_i32, c_i64, c_i64, c_i64, c_i64, c_i64, c_vp, c_vp, c_vp, c_vp, c_vp, c_sz,
                                c_vp]
        L.id_select_noalloc.argtypes = [c_vp, c_i32, c_i64, c_i64, c_i64, c_i64, c_i64, c_vp, c_vp, c_vp, c_vp, c_vp]
        L.id_select_noalloc.restype = c_i32
        L.ids_select_plan_info.argtypes = [c_i64, c_i64, c_i64, c_vp]
        L.ids_select_plan_info.restype = c_i32
        L.ids_tune_set.argtypes = [ctypes.c_char_p, c_i64]
        L.ids_tune_set.restype = c_i32
        L.ids_tune_get.argtypes = [ctypes.c_char_p, P(c_i64)]
        L.ids_tune_get.restype = c_i32
        L.ids_stream_read.argtypes = [c_vp, c_sz, c_vp, c_vp]
        L.ids_stream_read.restype = c_i32
        L.ids_set_wait_limit.argtypes = [c_i64]
        L.ids_set_wait_limit.restype = None
        L.ids_finalize.argtypes = []
        L.ids_finalize.restype = None
        L.ids_tensor_workspace_size.argtypes = [c_i32, c_vp, c_i64, c_i64, c_i64, c_i64, P(c_sz)]
        L.tensor_id.argtypes = [c_i32, c_vp, c_i64, c_vp, c_vp, c_vp, c_i64, c_i64, c_i64, c_vp, c_u64, c_vp, c_vp, c_vp,
                                c_vp, c_vp, c_vp, c_vp, c_sz, c_vp]
        L.ids_tensor_csc_workspace_size.argtypes = [c_i32, c_vp, c_i64, c_i64, c_i64, c_i64, P(c_sz)]
        L.ids_tensor_csc_workspace_size.restype = c_i32
        L.tensor_id_csc.argtypes = [c_i32, c_vp, c_i64, c_vp, c_vp, c_vp, c_vp, c_i64, c_i64, c_i64, c_vp, c_u64,
                                    c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_sz, c_vp]
        L.tensor_id_csc.restype = c_i32
        L.ids_batched_plan_size.argtypes = [c_i64, P(c_sz)]
        L.ids_batched_plan.argtypes = [c_i64, c_vp, c_vp, c_i64, c_i64, c_i64, c_vp, c_sz, P(c_sz), c_vp]
        L.id_batched.argtypes = [c_i64, c_vp, c_vp, c_vp, c_i64, c_i64, c_i64, c_u64, ctypes.c_double, c_vp, c_vp, c_vp,
                                 c_vp, c_vp, c_vp, c_vp, c_sz, c_vp]
        L.ids_batched_graph_create.argtypes = [c_i64, c_vp, c_vp, c_vp, c_i64, c_i64, c_i64, c_u64, ctypes.c_double,
                                               c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_sz, P(c_vp)]
        L.ids_batched_graph_launch.argtypes = [c_vp, c_vp]
        L.ids_batched_graph_destroy.argtypes = [c_vp]
        L.ids_batched_graph_destroy.restype = None
        for fn in ("ids_batched_plan_size", "ids_batched_plan", "id_batched", "ids_batched_graph_create",
                   "ids_batched_graph_launch"):
            getattr(L, fn).restype = c_i32
        L.ids_profile_enable.argtypes = [c_i32]
        L.ids_profile_enable.restype = None
        L.ids_profile_stages.argtypes = [ctypes.c_char_p]
        L.ids_profile_stages.restype = c_i32
        L.ids_profile_read.argtypes = [ctypes.c_char_p, P(ctypes.c_double), P(c_i64)]
        L.ids_profile_read.restype = c_i32
        L.ids_profile_reset.argtypes = []
        L.ids_profile_reset.restype = None
        L.ids_status_string.restype = ctypes.c_char_p
        L.ids_status_string.argtypes = [c_i32]
        L.ids_last_error.restype = ctypes.c_char_p
        L.ids_last_error.argtypes = []
        for fn in ("ids_sketch_workspace_size", "id_sketch", "id_project", "ids_select_workspace_size",
                   "id_select", "ids_tensor_workspace_size", "tensor_id"):
            getattr(L, fn).restype = c_i32
        _lib = L
        # release the library's streams and events before the HIP runtime goes
        atexit.register(L.ids_finalize)
    return _lib


def _check(status: int, what: str):
    if status != 0:
        L = lib()
        raise IdsError(f"{what}: {L.ids_status_string(status).decode()} -- {L.ids_last_error().decode()}")


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise IdsError("idsketch needs a ROCm GPU (torch.cuda.is_available() is False)")
    return torch


def _stream(torch, stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return c_vp(s.cuda_stream)


def _dt(t) -> int:
    import torch
    if t.dtype == torch.float64:
        return F64
    if t.dtype == torch.float32:
        return F32
    if t.dtype == torch.bfloat16:
        return BF16
    raise IdsError(f"unsupported dtype {t.dtype}")


def _tdt(code: int):
    import torch
    return {F64: torch.float64, F32: torch.float32, BF16: torch.bfloat16}[code]


def _workspace(torch, nbytes: int, device, stream=None):
    if nbytes == 0:
        return None, 0
    buf = torch.empty(int(nbytes) + 256, dtype=torch.uint8, device=device)
    if stream is not None:
        buf.record_stream(stream)  # keep the block reserved until `stream` is done
    ptr = buf.data_ptr()
    pad = (-ptr) % 256
    return (buf, ptr + pad), int(nbytes)


def _matrix_desc(A):
    """Dense torch matrix (row-major, unit column stride) or CSR tuple
    (rowptr int64, colind int32, val float64, n)."""
    if isinstance(A, tuple):
        rowptr, colind, val, n = A
        assert rowptr.dtype.is_floating_point is False
        d = IdsMatrix(CSR, F64, rowptr.numel() - 1, int(n), 0, val.numel(), c_vp(val.data_ptr()),
                      c_vp(rowptr.data_ptr()), c_vp(colind.data_ptr()))
        return d, val.device
    if A.dim() != 2 or A.stride(1) != 1:
        raise IdsError("dense A must be a 2-D tensor with unit column stride (row-major)")
    d = IdsMatrix(DENSE, _dt(A), A.shape[0], A.shape[1], A.stride(0), 0, c_vp(A.data_ptr()), None, None)
    return d, A.device


def check_status(status, what: str = "idsketch"):
    """Wait for the stream and raise IdsError if a device status word (a
    tensor of int32 codes, e.g. the "status" entry of a result) reports
    IDS_ETIMEOUT or IDS_ENONFINITE.  IDS_ERANKDEF is not an error: k_eff
    tells the rank reached."""
    torch = _torch()
    torch.cuda.synchronize(status.device)
    codes = set(int(c) for c in status.cpu().reshape(-1).tolist())
    for bad in (ETIMEOUT, ENONFINITE):
        if bad in codes:
            L = lib()
            raise IdsError(f"{what}: device status {L.ids_status_string(bad).decode()}")
    return codes


def select_plan_info(l: int, n: int, k: int) -> dict:
    """How id_select runs an l x n, rank-k shape (kernel family, candidate
    exchange, workgroups, publishers per step); host only."""
    info = (c_i32 * 4)()
    _check(lib().ids_select_plan_info(l, n, k, ctypes.cast(info, c_vp)), "ids_select_plan_info")
    return {"family": ["grouped_lanes", "row_bands", "column_steps"][info[0]],
            "exchange": ["speculative", "owner", "none"][info[1]], "workgroups": info[2], "publishers": info[3]}


def stream_read(buf, checksum, stream=None):
    """Read every byte of the device tensor `buf` once (measurement utility);
    the XOR of its 32-bit words goes to the int32 device tensor `checksum`."""
    torch = _torch()
    nbytes = buf.numel() * buf.element_size()
    _check(lib().ids_stream_read(c_vp(buf.data_ptr()), nbytes, c_vp(checksum.data_ptr()), _stream(torch, stream)),
           "ids_stream_read")


def tune_set(key: str, value: int | None):
    """Override a launch-shape knob (None: back to the tuned table's value)."""
    _check(lib().ids_tune_set(key.encode(), -1 if value is None else int(value)), "ids_tune_set")


def tune_get(key: str) -> int:
    v = c_i64(0)
    _check(lib().ids_tune_get(key.encode(), ctypes.byref(v)), "ids_tune_get")
    return v.value


def set_wait_limit(polls: int | None = None):
    """Polls before a device-wide wait of the pivoted QR gives up (None: the
    default; 0: give up at once -- a forced test of the timeout path)."""
    lib().ids_set_wait_limit(-1 if polls is None else int(polls))


def finalize():
    """Release the library's streams and events (also done at exit)."""
    lib().ids_finalize()


def profile_enable(on: bool = True):
    """Record HIP events around every stage of subsequent calls."""
    lib().ids_profile_enable(1 if on else 0)


def profile_stages(stages: str | None = None):
    """Restrict recording to the named stages (comma-separated); None: all."""
    _check(lib().ids_profile_stages(stages.encode() if stages else None), "ids_profile_stages")


def profile_read(stage: str):
    """(total milliseconds, number of launches) recorded for a stage."""
    ms = ctypes.c_double(0.0)
    cnt = c_i64(0)
    _check(lib().ids_profile_read(stage.encode(), ctypes.byref(ms), ctypes.byref(cnt)), "ids_profile_read")
    return ms.value, cnt.value


def profile_reset():
    lib().ids_profile_reset()


def id_sketch(A, l1: int, l: int | None = None, *, seed: int = 0, tag: int = 0, G=None, acc: int | None = None,
              fullrank=None, stream=None, check_finite=None, deterministic: bool = False):
    """Y = (G) S A, returned as an l x n view of a column-major buffer.
    check_finite: an int32 device tensor that receives IDS_OK or
    IDS_ENONFINITE from a scan of Y (flag IDS_CHECK_FINITE).
    deterministic: CSR entries summed in row order (flag IDS_DETERMINISTIC)."""
    torch = _torch()
    desc, dev = _matrix_desc(A)
    if l is None:
        l = l1
    if acc is None:
        acc = F64 if desc.dtype == F64 else F32
    flags = 0
    pi = x = None
    if fullrank is not None:
        pi, x = fullrank
        flags |= HASH_FULLRANK
    if check_finite is not None:
        flags |= CHECK_FINITE
    if deterministic:
        flags |= DETERMINISTIC
    cfg = IdsSketchCfg(l1, l, seed, tag, flags, acc, acc, c_vp(G.data_ptr()) if G is not None else None,
                       c_vp(pi.data_ptr()) if pi is not None else None, c_vp(x.data_ptr()) if x is not None else None,
                       _ptr(check_finite))
    if G is not None and l < l1:   # G None: drawn on the device from the stream (seed, tag | 2^63)
        if _dt(G) != acc or tuple(G.shape) != (l, l1) or not G.is_contiguous():
            raise IdsError("G must be a contiguous l x l1 tensor of the accumulation dtype")
    nbytes = c_sz(0)
    _check(lib().ids_sketch_workspace_size(ctypes.byref(desc), ctypes.byref(cfg), ctypes.byref(nbytes)),
           "ids_sketch_workspace_size")
    ws, wsb = _workspace(torch, nbytes.value, dev, stream)
    Yb = torch.empty((desc.n, l), dtype=_tdt(acc), device=dev)
    _check(lib().id_sketch(ctypes.byref(desc), ctypes.byref(cfg), c_vp(Yb.data_ptr()), acc, l,
                           c_vp(ws[1]) if ws else None, wsb, _stream(torch, stream)), "id_sketch")
    return Yb.t()


def id_project(G, Y1, stream=None):
    """Y = G Y1 (G l x q, Y1 q x n, both row-major), returned l x n column-major."""
    torch = _torch()
    l, q = G.shape
    q2, n = Y1.shape
    if q2 != q or G.dtype != Y1.dtype or not G.is_contiguous() or Y1.stride(1) != 1:
        raise IdsError("shape/dtype/layout mismatch")
    Yb = torch.empty((n, l), dtype=G.dtype, device=G.device)
    _check(lib().id_project(_dt(G), l, q, n, c_vp(G.data_ptr()), c_vp(Y1.data_ptr()), Y1.stride(0),
                            c_vp(Yb.data_ptr()), l, _stream(torch, stream)), "id_project")
    return Yb.t()


def gaussian_sketch(A, Omega, stream=None):
    """Y = Omega A for a dense row-major A (m x n) and Omega (l x m, row-major,
    the dtype of A): the Gaussian sketch of the comparison method, returned as
    an l x n view of a column-major buffer."""
    torch = _torch()
    desc, dev = _matrix_desc(A)
    if isinstance(A, tuple):
        raise IdsError("the Gaussian sketch takes a dense A")
    l, m = Omega.shape
    if m != desc.m or _dt(Omega) != desc.dtype or not Omega.is_contiguous():
        raise IdsError("Omega must be a contiguous l x m tensor of the dtype of A")
    nbytes = c_sz(0)
    _check(lib().ids_gaussian_workspace_size(ctypes.byref(desc), l, ctypes.byref(nbytes)),
           "ids_gaussian_workspace_size")
    ws, wsb = _workspace(torch, nbytes.value, dev, stream)
    Yb = torch.empty((desc.n, l), dtype=A.dtype, device=dev)
    _check(lib().id_gaussian_sketch(ctypes.byref(desc), l, c_vp(Omega.data_ptr()), c_vp(Yb.data_ptr()), l,
                                    c_vp(ws[1]) if ws else None, wsb, _stream(torch, stream)), "id_gaussian_sketch")
    return Yb.t()


def _status(torch, device, n: int = 1):
    # every call path writes its status word(s) on the call's stream, so no
    # fill (which would run on torch's current stream) precedes it
    return torch.empty((n,), dtype=torch.int32, device=device)


def gaussian_id(A, k: int, Omega, stream=None):
    """The Gaussian-sketch ID (comparison method): Y = Omega A, then Algorithm 1."""
    Y = gaussian_sketch(A, Omega, stream=stream)
    st = _status(_torch(), Y.device)
    J, P, keff = id_select(Y, k, stream=stream, status=st)
    return dict(Y=Y, J=J, P=P, k_eff=keff, status=st)


def _ptr(t):
    return c_vp(t.data_ptr()) if t is not None else None


def id_select(Y, k: int, stream=None, status=None):
    """Algorithm 1 on a sketch Y (l x n, any strides).  Returns (J, P, k_eff)
    where J (int64[k]), P (float64 k x n) and k_eff (int64[1]) are device
    tensors; an int32 device tensor `status` (1 element), if given, receives
    the device status word."""
    torch = _torch()
    l, n = Y.shape
    nbytes = c_sz(0)
    _check(lib().ids_select_workspace_size(l, n, k, ctypes.byref(nbytes)), "ids_select_workspace_size")
    ws, wsb = _workspace(torch, nbytes.value, Y.device, stream)
    J = torch.empty(k, dtype=torch.int64, device=Y.device)
    P = torch.empty((k, n), dtype=torch.float64, device=Y.device)
    keff = torch.empty(1, dtype=torch.int64, device=Y.device)
    _check(lib().id_select(c_vp(Y.data_ptr()), _dt(Y), l, n, Y.stride(0), Y.stride(1), k, c_vp(J.data_ptr()),
                           c_vp(P.data_ptr()), c_vp(keff.data_ptr()), _ptr(status), c_vp(ws[1]) if ws else None, wsb,
                           _stream(torch, stream)), "id_select")
    return J, P, keff


def id_select_noalloc(Y, k: int, J, P, keff, status=None, stream=None):
    """id_select into caller-provided outputs (J int64[k], P float64 k x n,
    keff int64[1], optional status int32[1]) with the library's static
    scratch buffer: no device allocation anywhere in the call."""
    torch = _torch()
    l, n = Y.shape
    _check(lib().id_select_noalloc(c_vp(Y.data_ptr()), _dt(Y), l, n, Y.stride(0), Y.stride(1), k,
                                   c_vp(J.data_ptr()), c_vp(P.data_ptr()), c_vp(keff.data_ptr()), _ptr(status),
                                   _stream(torch, stream)), "id_select_noalloc")
    return J, P, keff


def matrix_id(A, k: int, l1: int, l: int | None = None, *, seed: int = 0, tag: int = 0, G=None,
              acc: int | None = None, fullrank=None, stream=None, check: bool = False,
              deterministic: bool = False):
    """Algorithm 2 (+ optional projection), then Algorithm 1.  Returns dict
    with Y, J, P, k_eff and the device status word ("status").  check=True
    waits for the result and raises on IDS_ETIMEOUT / IDS_ENONFINITE."""
    Y = id_sketch(A, l1, l, seed=seed, tag=tag, G=G, acc=acc, fullrank=fullrank, stream=stream,
                  deterministic=deterministic)
    st = _status(_torch(), Y.device)
    J, P, keff = id_select(Y, k, stream=stream, status=st)
    if check:
        check_status(st, "matrix_id")
    return dict(Y=Y, J=J, P=P, k_eff=keff, status=st)


def tensor_id(factors, lam, k: int, Jlen: int, *, seed: int = 0, l: int = 0, G=None, return_Y: bool = False,
              stream=None, check: bool = False):
    """Algorithm 3.  factors: list of I_n x R float64 device tensors with unit
    row stride (column-major, e.g. ``F.t().contiguous().t()``).  l > 0 with an
    l x Jlen float64 G adds the Gaussian second stage before the CPQR."""
    torch = _torch()
    N = len(factors)
    R = factors[0].shape[1]
    for f in factors:
        if f.dtype != torch.float64 or f.stride(0) != 1 or f.shape[1] != R:
            raise IdsError("factors must be float64, column-major (stride(0) == 1), I_n x R")
    dims = (c_i64 * N)(*[f.shape[0] for f in factors])
    ld = (c_i64 * N)(*[f.stride(1) for f in factors])
    fptr = (c_vp * N)(*[f.data_ptr() for f in factors])
    dev = factors[0].device
    if l and G is not None:   # G None: drawn on the device from the stream (seed, 0 | 2^63)
        if G.dtype != torch.float64 or tuple(G.shape) != (l, Jlen) or not G.is_contiguous():
            raise IdsError("G must be a contiguous float64 l x Jlen tensor when l > 0")
    nbytes = c_sz(0)
    _check(lib().ids_tensor_workspace_size(N, ctypes.cast(dims, c_vp), R, k, Jlen, l, ctypes.byref(nbytes)),
           "ids_tensor_workspace_size")
    ws, wsb = _workspace(torch, nbytes.value, dev, stream)
    Y = torch.empty((R, Jlen), dtype=torch.float64, device=dev) if return_Y else None
    J = torch.empty(k, dtype=torch.int64, device=dev)
    P = torch.empty((k, R), dtype=torch.float64, device=dev)
    lh = torch.empty(k, dtype=torch.float64, device=dev)
    keff = torch.empty(1, dtype=torch.int64, device=dev)
    st = _status(torch, dev)
    _check(lib().tensor_id(N, ctypes.cast(dims, c_vp), R, ctypes.cast(fptr, c_vp), ctypes.cast(ld, c_vp),
                           c_vp(lam.data_ptr()), k, Jlen, l, c_vp(G.data_ptr()) if (l and G is not None) else None,
                           seed,
                           c_vp(Y.data_ptr()) if Y is not None else None,
                           c_vp(J.data_ptr()), c_vp(P.data_ptr()), c_vp(lh.data_ptr()), c_vp(keff.data_ptr()),
                           _ptr(st), c_vp(ws[1]) if ws else None, wsb, _stream(torch, stream)), "tensor_id")
    if check:
        check_status(st, "tensor_id")
    out = dict(J=J, P=P, lambda_hat=lh, k_eff=keff, status=st)
    if Y is not None:
        out["Y"] = Y.t()
    return out


def tensor_id_csc(factors, lam, k: int, Jlen: int, *, seed: int = 0, l: int = 0, G=None, return_Y: bool = False,
                  stream=None, check: bool = False):
    """Algorithm 3 for factors with sparse columns.  factors: list of
    (colptr int64[R+1], rowind int32, val float64, I_n) device tensors, the
    compressed sparse columns of each I_n x R factor (rows ascending within a
    column).  Otherwise as tensor_id."""
    torch = _torch()
    N = len(factors)
    R = factors[0][0].numel() - 1
    for cp, ri, v, _ in factors:
        if cp.dtype != torch.int64 or ri.dtype != torch.int32 or v.dtype != torch.float64 or cp.numel() != R + 1:
            raise IdsError("CSC factors need int64 colptr[R+1], int32 rowind and float64 val")
    dims = (c_i64 * N)(*[int(f[3]) for f in factors])
    cps = (c_vp * N)(*[f[0].data_ptr() for f in factors])
    ris = (c_vp * N)(*[f[1].data_ptr() for f in factors])
    vs = (c_vp * N)(*[f[2].data_ptr() for f in factors])
    dev = factors[0][2].device
    if l and G is not None:
        if G.dtype != torch.float64 or tuple(G.shape) != (l, Jlen) or not G.is_contiguous():
            raise IdsError("G must be a contiguous float64 l x Jlen tensor when l > 0")
    nbytes = c_sz(0)
    _check(lib().ids_tensor_csc_workspace_size(N, ctypes.cast(dims, c_vp), R, k, Jlen, l, ctypes.byref(nbytes)),
           "ids_tensor_csc_workspace_size")
    ws, wsb = _workspace(torch, nbytes.value, dev, stream)
    Y = torch.empty((R, Jlen), dtype=torch.float64, device=dev) if return_Y else None
    J = torch.empty(k, dtype=torch.int64, device=dev)
    P = torch.empty((k, R), dtype=torch.float64, device=dev)
    lh = torch.empty(k, dtype=torch.float64, device=dev)
    keff = torch.empty(1, dtype=torch.int64, device=dev)
    st = _status(torch, dev)
    _check(lib().tensor_id_csc(N, ctypes.cast(dims, c_vp), R, ctypes.cast(cps, c_vp), ctypes.cast(ris, c_vp),
                               ctypes.cast(vs, c_vp), c_vp(lam.data_ptr()), k, Jlen, l,
                               c_vp(G.data_ptr()) if (l and G is not None) else None, seed,
                               c_vp(Y.data_ptr()) if Y is not None else None, c_vp(J.data_ptr()),
                               c_vp(P.data_ptr()), c_vp(lh.data_ptr()), c_vp(keff.data_ptr()), _ptr(st),
                               c_vp(ws[1]) if ws else None, wsb, _stream(torch, stream)), "tensor_id_csc")
    if check:
        check_status(st, "tensor_id_csc")
    out = dict(J=J, P=P, lambda_hat=lh, k_eff=keff, status=st)
    if Y is not None:
        out["Y"] = Y.t()
    return out


class BatchedPlan:
    """Device-resident descriptors of a batch of problems (see ids_batched_plan)."""

    def __init__(self, m, n, k, l, l1max, buf, ws_bytes):
        import numpy as np
        self.m = np.ascontiguousarray(m, dtype=np.int64)
        self.n = np.ascontiguousarray(n, dtype=np.int64)
        self.k, self.l, self.l1max = int(k), int(l), int(l1max)
        self.buf = buf
        self.ws_bytes = int(ws_bytes)
        self.nprob = int(self.m.shape[0])
        self.a_off = np.concatenate([[0], np.cumsum(self.m * self.n)])
        self.p_off = np.concatenate([[0], np.cumsum(self.k * self.n)])
        self.y_off = np.concatenate([[0], np.cumsum(self.l * self.n)])


def batched_plan(m, n, k: int, l: int, l1max: int, device="cuda:0", stream=None) -> BatchedPlan:
    import numpy as np
    torch = _torch()
    m = np.ascontiguousarray(m, dtype=np.int64)
    n = np.ascontiguousarray(n, dtype=np.int64)
    nprob = m.shape[0]
    nb = c_sz(0)
    _check(lib().ids_batched_plan_size(nprob, ctypes.byref(nb)), "ids_batched_plan_size")
    buf = torch.empty(nb.value, dtype=torch.uint8, device=device)
    wsb = c_sz(0)
    _check(lib().ids_batched_plan(nprob, c_vp(m.ctypes.data), c_vp(n.ctypes.data), k, l, l1max,
                                  c_vp(buf.data_ptr()), nb.value, ctypes.byref(wsb), _stream(torch, stream)),
           "ids_batched_plan")
    return BatchedPlan(m, n, k, l, l1max, buf, wsb.value)


def id_batched(plan: BatchedPlan, A, G, seed: int = 0, tol: float = 0.0, stream=None, return_Y: bool = False):
    """Batched mixed-precision ID.  A: flat bfloat16 device tensor of all A_p
    (row-major, back to back); G: l x l1max bfloat16.  Returns dict with J
    (nprob x k), P (flat float64, P_p = P[p_off[p]:p_off[p+1]].view(k, n_p)),
    k_eff (nprob) and, if asked, Y (flat float32, Y_p column-major l x n_p).
    tol > 0: fixed accuracy, problem p stops once |r_tt| <= tol |r_11|."""
    torch = _torch()
    if A.dtype != torch.bfloat16 or (G is not None and G.dtype != torch.bfloat16):
        raise IdsError("A and G must be bfloat16")
    if G is not None and (tuple(G.shape) != (plan.l, plan.l1max) or not G.is_contiguous()):
        raise IdsError("G must be a contiguous l x l1max tensor (or None: drawn on the device)")
    if A.numel() < int(plan.a_off[-1]):
        raise IdsError("A is smaller than the batch")
    dev = A.device
    ws, wsb = _workspace(torch, plan.ws_bytes, dev, stream)
    J = torch.empty((plan.nprob, plan.k), dtype=torch.int64, device=dev)
    P = torch.empty(int(plan.p_off[-1]), dtype=torch.float64, device=dev)
    keff = torch.empty(plan.nprob, dtype=torch.int64, device=dev)
    st = _status(torch, dev, plan.nprob)
    _check(lib().id_batched(plan.nprob, c_vp(plan.m.ctypes.data), c_vp(plan.n.ctypes.data),
                            c_vp(plan.buf.data_ptr()), plan.k, plan.l, plan.l1max, seed, float(tol),
                            c_vp(A.data_ptr()),
                            _ptr(G), c_vp(J.data_ptr()), c_vp(P.data_ptr()), c_vp(keff.data_ptr()),
                            _ptr(st), c_vp(ws[1]), wsb, _stream(torch, stream)), "id_batched")
    out = dict(J=J, P=P, k_eff=keff, status=st)
    if return_Y:
        # Y is the first region of the workspace (FP32, Y_p column-major l x n_p)
        ny = int(plan.y_off[-1])
        start = ws[1] - ws[0].data_ptr()
        out["Y"] = ws[0][start:start + 4 * ny].view(torch.float32).clone()
    return out


class BatchedGraph:
    """One id_batched call recorded into a HIP graph (ids_batched_graph_create);
    launch() replays the whole batch on the current stream.  It owns its
    outputs (J, P, k_eff, status) and workspace, which every replay
    overwrites."""

    def __init__(self, plan: BatchedPlan, A, G, seed: int, tol: float):
        torch = _torch()
        dev = A.device
        self.plan, self.A, self.G = plan, A, G
        self.ws, self.wsb = _workspace(torch, plan.ws_bytes, dev)
        self.J = torch.empty((plan.nprob, plan.k), dtype=torch.int64, device=dev)
        self.P = torch.empty(int(plan.p_off[-1]), dtype=torch.float64, device=dev)
        self.k_eff = torch.empty(plan.nprob, dtype=torch.int64, device=dev)
        self.status = _status(torch, dev, plan.nprob)
        h = c_vp()
        _check(lib().ids_batched_graph_create(plan.nprob, c_vp(plan.m.ctypes.data), c_vp(plan.n.ctypes.data),
                                              c_vp(plan.buf.data_ptr()), plan.k, plan.l, plan.l1max, seed,
                                              float(tol), c_vp(A.data_ptr()), _ptr(G),
                                              c_vp(self.J.data_ptr()), c_vp(self.P.data_ptr()),
                                              c_vp(self.k_eff.data_ptr()), _ptr(self.status), c_vp(self.ws[1]),
                                              self.wsb, ctypes.byref(h)), "ids_batched_graph_create")
        self.handle = h

    def launch(self, stream=None):
        torch = _torch()
        _check(lib().ids_batched_graph_launch(self.handle, _stream(torch, stream)), "ids_batched_graph_launch")
        return dict(J=self.J, P=self.P, k_eff=self.k_eff, status=self.status)

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            lib().ids_batched_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def batched_graph(plan: BatchedPlan, A, G, seed: int = 0, tol: float = 0.0) -> BatchedGraph:
    """Record the batched ID of `plan` on A, G into a HIP graph (see BatchedGraph)."""
    if A.dtype.itemsize != 2 or (G is not None and G.dtype.itemsize != 2):
        raise IdsError("A and G must be bfloat16")
    return BatchedGraph(plan, A, G, seed, tol)
