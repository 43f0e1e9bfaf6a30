"""Interpolative (ID) and CUR decompositions on AMD MI355X (gfx950).

A thin ctypes binding over ``libidcur.so`` (C ABI in ``include/idcur.h``): it
allocates device buffers with torch, passes raw pointers and the current HIP
stream, and trims the outputs to the rank the device produced. Every step of
the computation runs in the library's HIP kernels; there is no host fallback
and importing this package fails if the library has not been built
(``python -m paper_1412_8447_amd.build``).

Entry points (names as in the C ABI, Section references to Voronin &
Martinsson, "Efficient Algorithms for CUR and Interpolative Matrix
Decompositions"):

* ``id_col``        column ID, Section 2.3 / Algorithm 1 (Algorithm 4 with p >= 0)
* ``id_row``        row ID, the column ID of A^T (remark closing Section 2.3)
* ``id_two_sided``  two-sided ID, Section 2.4 / Algorithm 2
* ``cur``           CUR-ID, Section 3 / Algorithm 3
* ``gaussian``      the Philox4x32-10 Gaussian sketch matrix of Section 5.1
* ``sketch``        the randomized sketch Y = Omega A (Section 5.1) with the power
                    steps of Section 5.3, in FP32 or on BF16 / FP16 matrix cores
* ``BatchedID``     adaptive-rank column IDs of many FP32 blocks in one persistent
                    launch (Section 3's tolerance variant on the sketch of Section
                    5.1), capturable in a graph, with a launch autotuner
"""
from __future__ import annotations

import atexit
import ctypes
import os
from dataclasses import dataclass
from typing import Optional

import torch

from .flops import flop_model  # noqa: F401  (host-side accounting, no compute)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libidcur.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build it with `python -m paper_1412_8447_amd.build` "
        "(there is no fallback implementation)"
    )

_lib = ctypes.CDLL(LIB_PATH)

# ---------------------------------------------------------------------------
# C declarations
# ---------------------------------------------------------------------------
OK, EINVAL, EDTYPE, EWORKSPACE, EHIP, ERANKCAP, ENONFINITE, ETIMEOUT = 0, -1, -2, -3, -4, -5, -6, -7
F64, F32 = 0, 1
PREC_NATIVE, PREC_BF16, PREC_FP16 = 0, 1, 2
NORMS_DOWNDATE, NORMS_EXACT = 0, 1
OP_ID_COL, OP_ID_ROW, OP_TWO_SIDED, OP_CUR, OP_SKETCH, OP_SKETCH_ROW = 0, 1, 2, 3, 4, 5
SKETCH_GAUSSIAN, SKETCH_SRHT = 0, 1

STATUS_NAMES = {OK: "OK", EINVAL: "EINVAL", EDTYPE: "EDTYPE", EWORKSPACE: "EWORKSPACE", EHIP: "EHIP",
                ERANKCAP: "ERANKCAP", ENONFINITE: "ENONFINITE", ETIMEOUT: "ETIMEOUT"}


class Opts(ctypes.Structure):
    _fields_ = [
        ("k", ctypes.c_int32),
        ("kmax", ctypes.c_int32),
        ("tol", ctypes.c_double),
        ("rank_tol", ctypes.c_double),
        ("p", ctypes.c_int32),
        ("q", ctypes.c_int32),
        ("seed", ctypes.c_uint64),
        ("omega", ctypes.c_void_p),
        ("prec", ctypes.c_int32),
        ("norms", ctypes.c_int32),
        ("sketch", ctypes.c_int32),
        ("srht_signs", ctypes.c_void_p),
        ("srht_rows", ctypes.c_void_p),
        ("u_correct", ctypes.c_int32),
        ("t_reg", ctypes.c_double),
        ("t_svd", ctypes.c_double),
    ]


_vp, _i32, _i64, _sz, _u64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t, ctypes.c_uint64
_lib.idcur_opts_default.argtypes = [ctypes.POINTER(Opts)]
_lib.idcur_opts_default.restype = None
_lib.idcur_create.argtypes = [ctypes.POINTER(_vp), _vp]
_lib.idcur_set_stream.argtypes = [_vp, _vp]
_lib.idcur_destroy.argtypes = [_vp]
_lib.idcur_last_error.argtypes = [_vp]
_lib.idcur_last_error.restype = ctypes.c_char_p
_lib.idcur_sync_status.argtypes = [_vp]
_lib.idcur_workspace_bytes.argtypes = [_vp, _i32, _i32, _i64, _i64, ctypes.POINTER(Opts), ctypes.POINTER(_sz)]
_common = [_vp, _i32, _i64, _i64, _vp, _i64, ctypes.POINTER(Opts), _vp, _sz, _vp]
_lib.idcur_id_col.argtypes = _common + [_vp, _vp, _i64]
_lib.idcur_id_col_noalloc.argtypes = [_vp, _i32, _i64, _i64, _vp, _i64, ctypes.POINTER(Opts), _vp, _vp, _vp, _i64]
_lib.idcur_id_col_noalloc.restype = ctypes.c_int
_lib.idcur_id_col_csc_workspace_bytes.argtypes = [_vp, _i32, _i64, _i64, _i64, ctypes.POINTER(Opts),
                                                  ctypes.POINTER(_sz)]
_lib.idcur_id_col_csc.argtypes = [_vp, _i32, _i64, _i64, _i64, _vp, _vp, _vp, ctypes.POINTER(Opts), _vp, _sz, _vp,
                                  _vp, _vp, _i64]
_lib.idcur_cur_csc_workspace_bytes.argtypes = [_vp, _i32, _i64, _i64, _i64, ctypes.POINTER(Opts), ctypes.POINTER(_sz)]
_lib.idcur_cur_csc_workspace_bytes.restype = ctypes.c_int
_lib.idcur_cur_csc.argtypes = [_vp, _i32, _i64, _i64, _i64, _vp, _vp, _vp, ctypes.POINTER(Opts), _vp, _sz, _vp, _vp,
                               _vp, _vp, _i64, _vp, _i64, _vp, _i64]
_lib.idcur_cur_csc.restype = ctypes.c_int
_lib.idcur_id_row.argtypes = _common + [_vp, _vp, _i64]
_lib.idcur_id_two_sided.argtypes = _common + [_vp, _vp, _i64, _vp, _vp, _i64]
_lib.idcur_cur.argtypes = _common + [_vp, _vp, _vp, _i64, _vp, _i64, _vp, _i64]
_lib.idcur_gaussian.argtypes = [_vp, _i32, _i64, _i64, _u64, _u64, _vp, _i64]
_lib.idcur_id_col_batched_workspace_bytes.argtypes = [_vp, _i32, _i32, _i32, _i32, ctypes.POINTER(Opts), ctypes.POINTER(_sz)]
_batched_args = [_vp, _i32, _i32, _i32, _i32, _vp, _vp, _vp, _vp, ctypes.POINTER(Opts), _vp, _sz, _vp, _vp, _vp, _vp]
_lib.idcur_id_col_batched.argtypes = _batched_args
_lib.idcur_id_col_batched_autotune.argtypes = _batched_args + [ctypes.POINTER(_i32)]
_lib.idcur_id_col_batched_set_variant.argtypes = [_vp, _i32]
_lib.idcur_sketch.argtypes = [_vp, _i32, _i32, _i64, _i64, _vp, _i64, ctypes.POINTER(Opts), _vp, _sz, _vp, _i64]
_lib.idcur_error_workspace_bytes.argtypes = [_vp, _i32, _i32, _i64, _i64, _i32, ctypes.POINTER(_sz)]
_lib.idcur_id_error.argtypes = [_vp, _i32, _i64, _i64, _vp, _i64, _vp, _vp, _i64, _vp, _i32, _vp, _sz, _vp]
_lib.idcur_cur_error.argtypes = [_vp, _i32, _i64, _i64, _vp, _i64, _vp, _i64, _vp, _i64, _vp, _i64, _vp, _i32, _vp,
                                 _sz, _vp]
_lib.idcur_id_col_backward_workspace_bytes.argtypes = [_vp, _i32, _i64, _i64, _i32, _i32, _i32, ctypes.POINTER(_sz)]
_lib.idcur_id_col_backward.argtypes = [_vp, _i32, _i64, _i64, _vp, _i64, _vp, _i32, _vp, _i32, _vp, _i64,
                                       ctypes.c_double, _vp, _i64, _vp, _sz]
_lib.idcur_id_col_batched_backward_workspace_bytes.argtypes = [_vp, _i32, _i32, _i32, _i32, ctypes.POINTER(Opts),
                                                                ctypes.POINTER(_sz)]
_lib.idcur_id_col_batched_backward.argtypes = [_vp, _i32, _i32, _i32, _i32, _vp, _vp, _vp, _vp, ctypes.POINTER(Opts),
                                               _vp, _vp, _vp, _vp, ctypes.c_double, _vp, _vp, _vp, _sz]
_lib.idcur_timing_enable.argtypes = [_vp, _i32]
_lib.idcur_timing_read.argtypes = [_vp, ctypes.c_char_p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_i32)]
for _f in ("idcur_error_workspace_bytes", "idcur_id_error", "idcur_cur_error", "idcur_id_col_backward_workspace_bytes",
           "idcur_id_col_backward", "idcur_id_col_batched_backward_workspace_bytes", "idcur_id_col_batched_backward",
           "idcur_timing_enable", "idcur_timing_read", "idcur_create", "idcur_set_stream", "idcur_destroy", "idcur_sync_status", "idcur_workspace_bytes",
           "idcur_id_col", "idcur_id_row", "idcur_id_two_sided", "idcur_cur", "idcur_gaussian", "idcur_sketch",
           "idcur_id_col_batched_workspace_bytes", "idcur_id_col_batched", "idcur_id_col_batched_autotune",
           "idcur_id_col_batched_set_variant"):
    getattr(_lib, _f).restype = ctypes.c_int

EXPORTED = ("idcur_opts_default", "idcur_create", "idcur_set_stream", "idcur_destroy", "idcur_last_error",
            "idcur_sync_status", "idcur_workspace_bytes", "idcur_id_col", "idcur_id_row", "idcur_id_two_sided",
            "idcur_cur", "idcur_gaussian", "idcur_timing_enable", "idcur_timing_read", "idcur_error_workspace_bytes",
            "idcur_id_error", "idcur_cur_error", "idcur_id_col_backward_workspace_bytes", "idcur_id_col_backward",
            "idcur_sketch", "idcur_id_col_batched_workspace_bytes", "idcur_id_col_batched",
            "idcur_id_col_batched_autotune", "idcur_id_col_batched_set_variant",
            "idcur_id_col_batched_backward_workspace_bytes", "idcur_id_col_batched_backward",
            "idcur_id_col_csc_workspace_bytes", "idcur_id_col_csc", "idcur_id_col_noalloc",
            "idcur_cur_csc_workspace_bytes", "idcur_cur_csc")

STAGES = ("omega", "pack", "sketch_gemm", "orth", "cpqr", "trsm", "gather", "row_id", "row_cpqr", "u_solve", "error", "backward",
          "batched", "srht", "spmm")


class IDCurError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


# ---------------------------------------------------------------------------
# Context (one per device, bound to torch's current stream at each call)
# ---------------------------------------------------------------------------
_ctx: dict = {}


def _context(device: torch.device) -> ctypes.c_void_p:
    idx = device.index if device.index is not None else torch.cuda.current_device()
    if idx not in _ctx:
        with torch.cuda.device(idx):
            h = _vp()
            st = _lib.idcur_create(ctypes.byref(h), _vp(torch.cuda.current_stream(idx).cuda_stream))
            if st != OK:
                raise IDCurError(st, "idcur_create failed")
            _ctx[idx] = h
    h = _ctx[idx]
    _lib.idcur_set_stream(h, _vp(torch.cuda.current_stream(idx).cuda_stream))
    return h


@atexit.register
def _teardown() -> None:
    """Destroy the contexts (status words, pooled events) at interpreter exit,
    after the work queued on their streams has finished."""
    for idx, h in list(_ctx.items()):
        try:
            _lib.idcur_sync_status(h)
            _lib.idcur_destroy(h)
        except Exception:  # pragma: no cover - best effort at exit
            pass
        _ctx.pop(idx, None)


def _check(h, st: int) -> None:
    if st != OK:
        raise IDCurError(st, _lib.idcur_last_error(h).decode())


def sync_status(device=None) -> int:
    """Synchronise and return the device status code (0 when clean); raises on
    device-side errors other than the rank cap."""
    dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
    h = _context(dev)
    st = _lib.idcur_sync_status(h)
    if st not in (OK, ERANKCAP):
        raise IDCurError(st, _lib.idcur_last_error(h).decode())
    return st


def _dtype_code(t: torch.Tensor) -> int:
    if t.dtype == torch.float32:
        return F32
    if t.dtype == torch.float64:
        return F64
    raise IDCurError(EDTYPE, f"unsupported dtype {t.dtype}")


def make_opts(k: int = 0, *, tol: float = 0.0, kmax: int = 0, p: int = -1, q: int = 0, seed: int = 0,
              omega: Optional[torch.Tensor] = None, rank_tol: float = 0.0, norms: str = "downdate",
              prec: str = "native", srht: Optional[tuple] = None, u_correct: bool = False,
              t_reg: float = 0.0, t_svd: float = 0.0) -> Opts:
    """Options of a decomposition call. ``srht = (rows, signs)`` selects the
    subsampled randomized Hadamard sketch with the given device tensors (rows:
    int32[l], distinct, below the padded order; signs: int8, one per sketched
    row), instead of the Gaussian one. ``u_correct`` makes a CUR call solve the
    error-corrected system U R = V* + C^+ E for U. ``t_reg`` in (0, 1) takes the
    Tikhonov-stabilized interpolation matrices of Section 4.1 (weight t_reg
    times |S11(1, 1)|); ``t_svd`` in (0, 1) the truncated-SVD ones (singular
    values of S11 below t_svd times the largest dropped)."""
    o = Opts()
    _lib.idcur_opts_default(ctypes.byref(o))
    o.k, o.kmax, o.tol, o.rank_tol = int(k), int(kmax), float(tol), float(rank_tol)
    o.p, o.q, o.seed = int(p), int(q), int(seed)
    o.omega = omega.data_ptr() if omega is not None else None
    o.norms = {"downdate": NORMS_DOWNDATE, "exact": NORMS_EXACT}[norms]
    o.prec = {"native": PREC_NATIVE, "bf16": PREC_BF16, "fp16": PREC_FP16}[prec]
    if srht is not None:
        rows, signs = srht
        for t, name, dt in ((rows, "srht rows", torch.int32), (signs, "srht signs", torch.int8)):
            if not t.is_cuda or t.dtype != dt or not t.is_contiguous():
                raise IDCurError(EINVAL, f"{name} must be a contiguous device tensor of {dt}")
        o.sketch = SKETCH_SRHT
        o.srht_rows, o.srht_signs = rows.data_ptr(), signs.data_ptr()
    o.u_correct = 1 if u_correct else 0
    o.t_reg = float(t_reg)
    o.t_svd = float(t_svd)
    return o


def workspace_bytes(op: int, A: torch.Tensor, opts: Opts) -> int:
    h = _context(A.device)
    n = ctypes.c_size_t(0)
    _check(h, _lib.idcur_workspace_bytes(h, op, _dtype_code(A), A.shape[0], A.shape[1], ctypes.byref(opts),
                                         ctypes.byref(n)))
    return int(n.value)


def _prep(A: torch.Tensor, omega):
    if not A.is_cuda:
        raise IDCurError(EINVAL, "A must be a device tensor")
    if A.dim() != 2 or A.stride(1) != 1:
        raise IDCurError(EINVAL, "A must be a 2-D row-major tensor (unit column stride)")
    if omega is not None:
        if not omega.is_cuda or omega.dtype != A.dtype or not omega.is_contiguous():
            raise IDCurError(EINVAL, "omega must be a contiguous device tensor of A's dtype")
    return _context(A.device)


def _mat(t: torch.Tensor, name: str, dtype=None) -> None:
    """A matrix argument: a 2-D device tensor with unit column stride (row r at
    data_ptr + r * stride(0)), of ``dtype`` when given."""
    if not t.is_cuda or t.dim() != 2 or (t.shape[1] > 1 and t.stride(1) != 1):
        raise IDCurError(EINVAL, f"{name} must be a 2-D row-major device tensor (unit column stride)")
    if dtype is not None and t.dtype != dtype:
        raise IDCurError(EINVAL, f"{name} must have dtype {dtype}")


def _idx(t: torch.Tensor, name: str) -> None:
    if not t.is_cuda or t.dtype != torch.int32 or not t.is_contiguous():
        raise IDCurError(EINVAL, f"{name} must be a contiguous int32 device tensor")


def _ws(h, op, A, o, workspace):
    need = workspace_bytes(op, A, o)
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(need, dtype=torch.uint8, device=A.device)
    return workspace


def sketch(A: torch.Tensor, k: int = 0, *, row: bool = False, workspace=None, **kw) -> torch.Tensor:
    """The sketch an ID call with the same options factors: Y = Omega A (or
    Omega A^T with ``row=True``), l = k + p rows, returned transposed as the
    library writes it (``Yt``: n x l, or m x l). Keyword options as
    :func:`make_opts` (``p >= 0`` required; ``prec`` selects the matrix-core
    input precision)."""
    h = _prep(A, kw.get("omega"))
    o = make_opts(k, **kw)
    m, n = A.shape
    l = (o.k if o.k > 0 else o.kmax) + o.p
    op = OP_SKETCH_ROW if row else OP_SKETCH
    ws = _ws(h, op, A, o, workspace)
    Yt = torch.empty(m if row else n, max(l, 1), dtype=A.dtype, device=A.device)
    _check(h, _lib.idcur_sketch(h, op, _dtype_code(A), m, n, A.data_ptr(), A.stride(0), ctypes.byref(o),
                                ws.data_ptr(), ws.numel(), Yt.data_ptr(), Yt.stride(0)))
    return Yt


@dataclass
class ColumnID:
    J: torch.Tensor          # int32 (n,)
    T: torch.Tensor          # (k, n-k)
    k: int
    kout: Optional[torch.Tensor] = None   # device int32 [k, 0]


@dataclass
class TwoSided:
    J: torch.Tensor
    T: torch.Tensor
    I: torch.Tensor
    Tr: torch.Tensor
    k: int
    k_row: int


@dataclass
class CUR:
    J: torch.Tensor
    I: torch.Tensor
    C: torch.Tensor
    U: torch.Tensor
    R: torch.Tensor
    k: int
    k_row: int
    kout: Optional[torch.Tensor] = None   # device int32 [k, k_row]


def id_col(A: torch.Tensor, k: int = 0, *, workspace=None, sync: bool = True, **kw) -> ColumnID:
    """Column ID A ~ A(:, J[:k]) [I T] P*. Keyword options as :func:`make_opts`."""
    h = _prep(A, kw.get("omega"))
    o = make_opts(k, **kw)
    m, n = A.shape
    kcap = o.k if o.k > 0 else o.kmax
    ws = _ws(h, OP_ID_COL, A, o, workspace)
    J = torch.empty(n, dtype=torch.int32, device=A.device)
    ldt = n
    T = torch.empty(max(kcap, 1), max(ldt, 1), dtype=A.dtype, device=A.device)
    kout = torch.zeros(2, dtype=torch.int32, device=A.device)
    _check(h, _lib.idcur_id_col(h, _dtype_code(A), m, n, A.data_ptr(), A.stride(0), ctypes.byref(o), ws.data_ptr(),
                                ws.numel(), kout.data_ptr(), J.data_ptr(), T.data_ptr(), max(ldt, 1)))
    if not sync:
        return ColumnID(J, T, -1, kout)
    sync_status(A.device)
    kk = int(kout[0].item())
    return ColumnID(J, T[:kk, : n - kk], kk, kout)


def id_col_noalloc(A: torch.Tensor, k: int = 0, *, out=None, sync: bool = True, **kw) -> ColumnID:
    """Column ID through idcur_id_col_noalloc: no workspace, the library's fixed
    scratch array instead. ``out`` = (J, T, kout) reuses caller buffers (J int32[n],
    T of A's dtype with n columns and at least k (kmax) rows, kout int32[2])."""
    h = _prep(A, kw.get("omega"))
    o = make_opts(k, **kw)
    m, n = A.shape
    kcap = o.k if o.k > 0 else o.kmax
    if out is None:
        J = torch.empty(n, dtype=torch.int32, device=A.device)
        T = torch.empty(max(kcap, 1), max(n, 1), dtype=A.dtype, device=A.device)
        kout = torch.zeros(2, dtype=torch.int32, device=A.device)
    else:
        J, T, kout = out
    ldt = T.shape[1]
    _check(h, _lib.idcur_id_col_noalloc(h, _dtype_code(A), m, n, A.data_ptr(), A.stride(0), ctypes.byref(o),
                                        kout.data_ptr(), J.data_ptr(), T.data_ptr(), max(ldt, 1)))
    if not sync:
        return ColumnID(J, T, -1, kout)
    sync_status(A.device)
    kk = int(kout[0].item())
    return ColumnID(J, T[:kk, : n - kk], kk, kout)


def id_col_csc(colptr: torch.Tensor, rowidx: torch.Tensor, vals: torch.Tensor, m: int, n: int, k: int = 0, *,
               workspace=None, sync: bool = True, **kw) -> ColumnID:
    """Column ID of a sparse m x n matrix in compressed sparse column form
    (colptr int64[n+1], rowidx int32[nnz], vals float32/float64[nnz], all on one
    device): the sketch Omega A read entry by entry, then the dense CPQR and T.
    Keyword options as :func:`make_opts` (p >= 0, q = 0)."""
    for t, name, dt in ((colptr, "colptr", torch.int64), (rowidx, "rowidx", torch.int32)):
        if t.dtype != dt or t.dim() != 1 or not t.is_contiguous() or t.device != vals.device:
            raise IDCurError(EINVAL, f"{name} must be a contiguous 1-D {dt} tensor on the device of vals")
    if vals.dim() != 1 or not vals.is_contiguous() or colptr.numel() != n + 1 or rowidx.numel() != vals.numel():
        raise IDCurError(EINVAL, "vals must be contiguous 1-D with rowidx's length; colptr needs n + 1 entries")
    h = _context(vals.device)
    omega = kw.get("omega")
    if omega is not None:
        _mat(omega, "omega", vals.dtype)
    o = make_opts(k, **kw)
    nnz = vals.numel()
    kcap = o.k if o.k > 0 else o.kmax
    nb = _sz(0)
    _check(h, _lib.idcur_id_col_csc_workspace_bytes(h, _dtype_code(vals), m, n, nnz, ctypes.byref(o), ctypes.byref(nb)))
    ws = workspace if workspace is not None else torch.empty(nb.value, dtype=torch.uint8, device=vals.device)
    J = torch.empty(n, dtype=torch.int32, device=vals.device)
    T = torch.empty(max(kcap, 1), max(n, 1), dtype=vals.dtype, device=vals.device)
    kout = torch.zeros(2, dtype=torch.int32, device=vals.device)
    _check(h, _lib.idcur_id_col_csc(h, _dtype_code(vals), m, n, nnz, colptr.data_ptr(), rowidx.data_ptr(),
                                    vals.data_ptr(), ctypes.byref(o), ws.data_ptr(), ws.numel(), kout.data_ptr(),
                                    J.data_ptr(), T.data_ptr(), max(n, 1)))
    if not sync:
        return ColumnID(J, T, -1, kout)
    sync_status(vals.device)
    kk = int(kout[0].item())
    return ColumnID(J, T[:kk, : n - kk], kk, kout)


def cur_csc(colptr: torch.Tensor, rowidx: torch.Tensor, vals: torch.Tensor, m: int, n: int, k: int = 0, *,
            workspace=None, sync: bool = True, **kw) -> CUR:
    """CUR-ID of a sparse m x n matrix in compressed sparse column form
    (idcur_cur_csc): the sparse column ID, C and R gathered from the stored
    entries, the row ID of C and U = V* R^+. Options as :func:`id_col_csc`."""
    for t, name, dt in ((colptr, "colptr", torch.int64), (rowidx, "rowidx", torch.int32)):
        if not t.is_cuda or t.dtype != dt or not t.is_contiguous():
            raise IDCurError(EINVAL, f"{name} must be a contiguous device tensor of {dt}")
    if not vals.is_cuda or not vals.is_contiguous() or vals.dtype not in (torch.float32, torch.float64):
        raise IDCurError(EINVAL, "vals must be a contiguous FP32 / FP64 device tensor")
    h = _context(vals.device)
    o = make_opts(k, **kw)
    kcap = o.k if o.k > 0 else o.kmax
    code = _dtype_code(vals)
    nnz = int(vals.numel())
    if workspace is None:
        nb = _sz(0)
        _check(h, _lib.idcur_cur_csc_workspace_bytes(h, code, m, n, nnz, ctypes.byref(o), ctypes.byref(nb)))
        workspace = torch.empty(max(int(nb.value), 1), dtype=torch.uint8, device=vals.device)
    dev = vals.device
    J = torch.empty(n, dtype=torch.int32, device=dev)
    I = torch.empty(m, dtype=torch.int32, device=dev)
    U = torch.empty(kcap, kcap, dtype=vals.dtype, device=dev)
    C = torch.empty(m, kcap, dtype=vals.dtype, device=dev)
    R = torch.empty(kcap, n, dtype=vals.dtype, device=dev)
    kout = torch.zeros(2, dtype=torch.int32, device=dev)
    _check(h, _lib.idcur_cur_csc(h, code, m, n, nnz, colptr.data_ptr(), rowidx.data_ptr(), vals.data_ptr(),
                                 ctypes.byref(o), workspace.data_ptr(), workspace.numel(), kout.data_ptr(), J.data_ptr(),
                                 I.data_ptr(), U.data_ptr(), kcap, C.data_ptr(), kcap, R.data_ptr(), n))
    if not sync:
        return CUR(J, I, C, U, R, -1, -1, kout)
    sync_status(dev)
    k1, k2 = (int(v) for v in kout.tolist())
    return CUR(J, I, C[:, :k1], U[:k1, :k2], R[:k2], k1, k2, kout)


def id_row(A: torch.Tensor, k: int = 0, *, workspace=None, sync: bool = True, **kw) -> ColumnID:
    """Row ID A ~ W A(I[:k], :), returned as ColumnID(J=I, T=Tr)."""
    h = _prep(A, kw.get("omega"))
    o = make_opts(k, **kw)
    m, n = A.shape
    kcap = o.k if o.k > 0 else o.kmax
    ws = _ws(h, OP_ID_ROW, A, o, workspace)
    I = torch.empty(m, dtype=torch.int32, device=A.device)
    ldt = m
    Tr = torch.empty(max(kcap, 1), max(ldt, 1), dtype=A.dtype, device=A.device)
    kout = torch.zeros(2, dtype=torch.int32, device=A.device)
    _check(h, _lib.idcur_id_row(h, _dtype_code(A), m, n, A.data_ptr(), A.stride(0), ctypes.byref(o), ws.data_ptr(),
                                ws.numel(), kout.data_ptr(), I.data_ptr(), Tr.data_ptr(), max(ldt, 1)))
    if not sync:
        return ColumnID(I, Tr, -1)
    sync_status(A.device)
    kk = int(kout[0].item())
    return ColumnID(I, Tr[:kk, : m - kk], kk)


def id_two_sided(A: torch.Tensor, k: int = 0, *, workspace=None, **kw) -> TwoSided:
    h = _prep(A, kw.get("omega"))
    o = make_opts(k, **kw)
    m, n = A.shape
    kcap = o.k if o.k > 0 else o.kmax
    ws = _ws(h, OP_TWO_SIDED, A, o, workspace)
    J = torch.empty(n, dtype=torch.int32, device=A.device)
    I = torch.empty(m, dtype=torch.int32, device=A.device)
    ldt, ldtr = n, m
    T = torch.empty(max(kcap, 1), max(ldt, 1), dtype=A.dtype, device=A.device)
    Tr = torch.empty(max(kcap, 1), max(ldtr, 1), dtype=A.dtype, device=A.device)
    kout = torch.zeros(2, dtype=torch.int32, device=A.device)
    _check(h, _lib.idcur_id_two_sided(h, _dtype_code(A), m, n, A.data_ptr(), A.stride(0), ctypes.byref(o),
                                      ws.data_ptr(), ws.numel(), kout.data_ptr(), J.data_ptr(), T.data_ptr(),
                                      max(ldt, 1), I.data_ptr(), Tr.data_ptr(), max(ldtr, 1)))
    sync_status(A.device)
    k1, k2 = (int(v) for v in kout.tolist())
    return TwoSided(J, T[:k1, : n - k1], I, Tr[:k2, : m - k2], k1, k2)


def cur(A: torch.Tensor, k: int = 0, *, workspace=None, sync: bool = True, out=None, **kw) -> CUR:
    """CUR-ID: C = A(:, J[:k]), R = A(I[:k], :), U = V* R^+."""
    h = _prep(A, kw.get("omega"))
    o = make_opts(k, **kw)
    m, n = A.shape
    kcap = o.k if o.k > 0 else o.kmax
    ws = _ws(h, OP_CUR, A, o, workspace)
    if out is None:
        out = dict(
            J=torch.empty(n, dtype=torch.int32, device=A.device),
            I=torch.empty(m, dtype=torch.int32, device=A.device),
            U=torch.empty(kcap, kcap, dtype=A.dtype, device=A.device),
            C=torch.empty(m, kcap, dtype=A.dtype, device=A.device),
            R=torch.empty(kcap, n, dtype=A.dtype, device=A.device),
            kout=torch.zeros(2, dtype=torch.int32, device=A.device),
        )
    J, I, U, C, R, kout = out["J"], out["I"], out["U"], out["C"], out["R"], out["kout"]
    _check(h, _lib.idcur_cur(h, _dtype_code(A), m, n, A.data_ptr(), A.stride(0), ctypes.byref(o), ws.data_ptr(),
                             ws.numel(), kout.data_ptr(), J.data_ptr(), I.data_ptr(), U.data_ptr(), kcap,
                             C.data_ptr(), kcap, R.data_ptr(), n))
    if not sync:
        return CUR(J, I, C, U, R, -1, -1, kout)
    sync_status(A.device)
    k1, k2 = (int(v) for v in kout.tolist())
    return CUR(J, I, C[:, :k1], U[:k1, :k2], R[:k2], k1, k2, kout)


def gaussian(rows: int, cols: int, seed: int, *, stream_id: int = 0, dtype=torch.float32,
             device="cuda") -> torch.Tensor:
    """Omega (rows x cols) from the Philox4x32-10 / Box-Muller definition."""
    out = torch.empty(rows, cols, dtype=dtype, device=device)
    h = _context(out.device)
    _check(h, _lib.idcur_gaussian(h, _dtype_code(out), rows, cols, seed, stream_id, out.data_ptr(), cols))
    return out


def timing_enable(enable: bool = True, device=None) -> None:
    """Switch the per-stage event timers on or off (clears previous marks)."""
    dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
    h = _context(dev)
    _check(h, _lib.idcur_timing_enable(h, 1 if enable else 0))


def timing_read(device=None) -> dict:
    """{stage: (total_ms, launches)} accumulated since timing_enable."""
    dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
    h = _context(dev)
    out = {}
    for s in STAGES:
        ms, cnt = ctypes.c_double(0.0), _i32(0)
        _check(h, _lib.idcur_timing_read(h, s.encode(), ctypes.byref(ms), ctypes.byref(cnt)))
        out[s] = (ms.value, cnt.value)
    return out


def _err_ws(which, A, kcap, workspace):
    h = _context(A.device)
    nb = ctypes.c_size_t(0)
    _check(h, _lib.idcur_error_workspace_bytes(h, which, _dtype_code(A), A.shape[0], A.shape[1], kcap,
                                               ctypes.byref(nb)))
    if workspace is None or workspace.numel() < nb.value:
        workspace = torch.empty(int(nb.value), dtype=torch.uint8, device=A.device)
    return h, workspace


def id_error(A: torch.Tensor, J: torch.Tensor, T: torch.Tensor, kout: torch.Tensor, kcap: int, *, workspace=None,
             out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Device [|A - C V*|_F^2, |A|_F^2] (float64) for the column ID (J, T)."""
    _mat(A, "A")
    _mat(T, "T", A.dtype)
    _idx(J, "J")
    _idx(kout, "kout")
    h, ws = _err_ws(0, A, kcap, workspace)
    if out is None:
        out = torch.zeros(2, dtype=torch.float64, device=A.device)
    _check(h, _lib.idcur_id_error(h, _dtype_code(A), A.shape[0], A.shape[1], A.data_ptr(), A.stride(0), J.data_ptr(),
                                  T.data_ptr(), T.stride(0), kout.data_ptr(), kcap, ws.data_ptr(), ws.numel(),
                                  out.data_ptr()))
    return out


def cur_error(A: torch.Tensor, C: torch.Tensor, U: torch.Tensor, R: torch.Tensor, kout: torch.Tensor, kcap: int, *,
              workspace=None, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Device [|A - C U R|_F^2, |A|_F^2] (float64)."""
    _mat(A, "A")
    for t, nm in ((C, "C"), (U, "U"), (R, "R")):
        _mat(t, nm, A.dtype)
    _idx(kout, "kout")
    h, ws = _err_ws(1, A, kcap, workspace)
    if out is None:
        out = torch.zeros(2, dtype=torch.float64, device=A.device)
    _check(h, _lib.idcur_cur_error(h, _dtype_code(A), A.shape[0], A.shape[1], A.data_ptr(), A.stride(0), C.data_ptr(),
                                   C.stride(0), U.data_ptr(), U.stride(0), R.data_ptr(), R.stride(0), kout.data_ptr(),
                                   kcap, ws.data_ptr(), ws.numel(), out.data_ptr()))
    return out


# ---------------------------------------------------------------------------
# Gradient of the column-ID reconstruction loss (skeleton frozen)
# ---------------------------------------------------------------------------
def backward_workspace_bytes(A: torch.Tensor, k: int, l: int = 0, sketched: bool = False) -> int:
    """Workspace bytes of :func:`id_col_backward` for A's shape and dtype, rank k
    and (when sketched) l sketch rows."""
    h = _prep(A, None)
    m, n = A.shape
    nb = ctypes.c_size_t(0)
    _check(h, _lib.idcur_id_col_backward_workspace_bytes(h, _dtype_code(A), m, n, int(k), int(l) if sketched else 0,
                                                         1 if sketched else 0, ctypes.byref(nb)))
    return int(nb.value)


def id_col_backward(A: torch.Tensor, J: torch.Tensor, T: torch.Tensor, k: int, *, omega: Optional[torch.Tensor] = None,
                    scale: float = 1.0, out: Optional[torch.Tensor] = None, workspace=None) -> torch.Tensor:
    """scale * dL/dA for L = |A(:,J2) - A(:,J1) T|_F^2 with J and Omega fixed and T
    the least-squares interpolation from Y = Omega A (or Y = A when omega is None)."""
    h = _prep(A, omega)
    m, n = A.shape
    l = int(omega.shape[0]) if omega is not None else 0
    nb = ctypes.c_size_t(0)
    _check(h, _lib.idcur_id_col_backward_workspace_bytes(h, _dtype_code(A), m, n, int(k), l,
                                                         1 if omega is not None else 0, ctypes.byref(nb)))
    if workspace is None or workspace.numel() < nb.value:
        workspace = torch.empty(int(nb.value), dtype=torch.uint8, device=A.device)
    if out is None:
        out = torch.empty(m, n, dtype=A.dtype, device=A.device)
    _idx(J, "J")
    _mat(T, "T", A.dtype)
    _check(h, _lib.idcur_id_col_backward(h, _dtype_code(A), m, n, A.data_ptr(), A.stride(0),
                                         omega.data_ptr() if omega is not None else None, l, J.data_ptr(), int(k),
                                         T.data_ptr(), T.stride(0), float(scale), out.data_ptr(), out.stride(0),
                                         workspace.data_ptr(), workspace.numel()))
    return out


class IDReconLoss(torch.autograd.Function):
    """L(A) = |A(:,J2) - A(:,J1) T|_F^2 of the rank-k column ID of A (T from the
    sketch Y = Omega A when omega is given, one pass, no power steps). The
    skeleton J chosen in the forward pass is frozen in the backward pass."""

    @staticmethod
    def forward(ctx, A, k, omega=None):
        p = int(omega.shape[0]) - int(k) if omega is not None else -1
        r = id_col(A, int(k), p=p, q=0, omega=omega)
        if r.k != int(k):
            raise IDCurError(EINVAL, f"rank deficiency: the column ID stopped at {r.k} < k")
        Tfull = r.T.as_strided((r.k, A.shape[1] - r.k), (r.T.stride(0), 1))
        err = id_error(A, r.J, Tfull, r.kout, r.k)
        ctx.save_for_backward(A, r.J, Tfull, omega if omega is not None else torch.empty(0, device=A.device))
        ctx.k = r.k
        ctx.sketched = omega is not None
        return err[0].clone()

    @staticmethod
    def backward(ctx, g):
        A, J, T, omega = ctx.saved_tensors
        dA = id_col_backward(A, J, T, ctx.k, omega=omega if ctx.sketched else None, scale=float(g))
        return dA, None, None


def recon_loss(A: torch.Tensor, k: int, omega: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Differentiable column-ID reconstruction loss (see IDReconLoss)."""
    return IDReconLoss.apply(A, k, omega)


# ---------------------------------------------------------------------------
# Batched adaptive-rank column ID (one persistent launch)
# ---------------------------------------------------------------------------
@dataclass
class BlockID:
    J: torch.Tensor   # int32 (n_b,)
    T: torch.Tensor   # (k_b, n_b - k_b)
    k: int


class BatchedID:
    """Column IDs of many FP32 blocks (each 2-D, row-major, n_b <= 512) in one
    persistent launch (idcur_id_col_batched). Tolerance mode with ``tol`` and the
    rank cap ``kmax``, or a fixed rank ``k``; oversampling ``p``.

    The plan owns every device array the call reads or writes (block pointers and
    sizes, outputs, workspace), so :meth:`run` only enqueues kernels on the
    current stream and can be captured in a graph (``torch.cuda.CUDAGraph``)."""

    def __init__(self, blocks, *, tol: float = 0.0, kmax: int = 0, k: int = 0, p: int = 8, seed: int = 0,
                 omega: Optional[torch.Tensor] = None, rank_tol: float = 0.0):
        if not blocks:
            raise IDCurError(EINVAL, "no blocks")
        dev = blocks[0].device
        for b in blocks:
            _mat(b, "block", torch.float32)
            if b.device != dev:
                raise IDCurError(EINVAL, "all blocks must be on one device")
        if omega is not None:
            _mat(omega, "omega", torch.float32)
            omega = omega.contiguous()
        self.h = _context(dev)
        self.device = dev
        self.blocks = list(blocks)
        self.omega = omega
        ms = [int(b.shape[0]) for b in blocks]
        ns = [int(b.shape[1]) for b in blocks]
        self.ms, self.ns = ms, ns
        self.nblk = len(blocks)
        self.mmax, self.nmax = max(ms), max(ns)
        self.opts = make_opts(k, tol=tol, kmax=kmax, p=p, seed=seed, omega=omega, rank_tol=rank_tol)
        self.kcap = k if k > 0 else kmax
        i32, i64 = torch.int32, torch.int64
        self.m = torch.tensor(ms, dtype=i32, device=dev)
        self.n = torch.tensor(ns, dtype=i32, device=dev)
        self.A = torch.tensor([b.data_ptr() for b in blocks], dtype=i64, device=dev)
        self.lda = torch.tensor([b.stride(0) for b in blocks], dtype=i64, device=dev)
        offj, offt, oj, ot = [], [], 0, 0
        for nb in ns:
            offj.append(oj)
            offt.append(ot)
            oj += nb
            ot += max(self.kcap, 1) * nb
        self.offj, self.offt = offj, offt
        self.Jbuf = torch.empty(oj, dtype=i32, device=dev)
        self.Tbuf = torch.zeros(ot, dtype=torch.float32, device=dev)
        self.Jp = torch.tensor([self.Jbuf.data_ptr() + 4 * o for o in offj], dtype=i64, device=dev)
        self.Tp = torch.tensor([self.Tbuf.data_ptr() + 4 * o for o in offt], dtype=i64, device=dev)
        self.ldt = torch.tensor(ns, dtype=i64, device=dev)
        self.kout = torch.zeros(self.nblk, dtype=i32, device=dev)
        nbytes = ctypes.c_size_t(0)
        _check(self.h, _lib.idcur_id_col_batched_workspace_bytes(self.h, F32, self.nblk, self.mmax, self.nmax,
                                                                 ctypes.byref(self.opts), ctypes.byref(nbytes)))
        self.ws = torch.empty(max(int(nbytes.value), 1), dtype=torch.uint8, device=dev)
        self._dbuf = None

    def _args(self):
        return (self.h, F32, self.nblk, self.mmax, self.nmax, self.m.data_ptr(), self.n.data_ptr(),
                self.A.data_ptr(), self.lda.data_ptr(), ctypes.byref(self.opts), self.ws.data_ptr(),
                self.ws.numel(), self.kout.data_ptr(), self.Jp.data_ptr(), self.Tp.data_ptr(), self.ldt.data_ptr())

    def run(self) -> None:
        """Enqueue the batched launch on the current stream (no synchronisation)."""
        _lib.idcur_set_stream(self.h, _vp(torch.cuda.current_stream(self.device).cuda_stream))
        _check(self.h, _lib.idcur_id_col_batched(*self._args()))

    def autotune(self) -> int:
        """Time every launch variant on this batch, keep the fastest for its size
        class in the context; returns the variant (results are left in place)."""
        _lib.idcur_set_stream(self.h, _vp(torch.cuda.current_stream(self.device).cuda_stream))
        v = _i32(-1)
        _check(self.h, _lib.idcur_id_col_batched_autotune(*self._args(), ctypes.byref(v)))
        return int(v.value)

    def backward(self, scale: float = 1.0) -> None:
        """Enqueue the gradient of every block's reconstruction loss
        |A_b(:,J2) - A_b(:,J1) T_b|_F^2 with the skeleton of the last :meth:`run`
        frozen (idcur_id_col_batched_backward; fixed-rank plans only), times
        ``scale``, into the plan's gradient buffers (see :meth:`grads`). Only
        enqueues kernels on the current stream, so it can be captured in a graph."""
        if self.kcap <= 0 or self.opts.k <= 0:
            raise IDCurError(EINVAL, "the batched backward differentiates fixed-rank plans (k > 0)")
        if self._dbuf is None:
            dev, i64 = self.device, torch.int64
            offd, o = [], 0
            for mb, nb in zip(self.ms, self.ns):
                offd.append(o)
                o += mb * nb
            self._offd = offd
            self._dbuf = torch.empty(max(o, 1), dtype=torch.float32, device=dev)
            self._dp = torch.tensor([self._dbuf.data_ptr() + 4 * x for x in offd], dtype=i64, device=dev)
            self._ldd = torch.tensor(self.ns, dtype=i64, device=dev)
            nbytes = ctypes.c_size_t(0)
            _check(self.h, _lib.idcur_id_col_batched_backward_workspace_bytes(
                self.h, F32, self.nblk, self.mmax, self.nmax, ctypes.byref(self.opts), ctypes.byref(nbytes)))
            self._wsb = torch.empty(max(int(nbytes.value), 1), dtype=torch.uint8, device=dev)
        _lib.idcur_set_stream(self.h, _vp(torch.cuda.current_stream(self.device).cuda_stream))
        _check(self.h, _lib.idcur_id_col_batched_backward(
            self.h, F32, self.nblk, self.mmax, self.nmax, self.m.data_ptr(), self.n.data_ptr(), self.A.data_ptr(),
            self.lda.data_ptr(), ctypes.byref(self.opts), self.kout.data_ptr(), self.Jp.data_ptr(), self.Tp.data_ptr(),
            self.ldt.data_ptr(), float(scale), self._dp.data_ptr(), self._ldd.data_ptr(), self._wsb.data_ptr(),
            self._wsb.numel()))

    def grads(self) -> list:
        """Synchronise and return the gradients of the last :meth:`backward`, one
        m_b x n_b view per block (copy them before the next call)."""
        if self._dbuf is None:
            raise IDCurError(EINVAL, "backward() has not been called")
        st = _lib.idcur_sync_status(self.h)
        if st != OK:
            raise IDCurError(st, _lib.idcur_last_error(self.h).decode())
        return [self._dbuf[o: o + mb * nb].view(mb, nb) for o, mb, nb in zip(self._offd, self.ms, self.ns)]

    def results(self) -> list:
        """Synchronise and return one BlockID per block (views into the plan's
        output buffers: copy them before the next run)."""
        st = _lib.idcur_sync_status(self.h)
        if st not in (OK, ERANKCAP):
            raise IDCurError(st, _lib.idcur_last_error(self.h).decode())
        ks = self.kout.tolist()
        out = []
        for b, kb in enumerate(ks):
            nb = self.ns[b]
            J = self.Jbuf[self.offj[b]: self.offj[b] + nb]
            Tfull = self.Tbuf[self.offt[b]: self.offt[b] + max(self.kcap, 1) * nb].view(max(self.kcap, 1), nb)
            out.append(BlockID(J, Tfull[:max(kb, 0), : nb - max(kb, 0)], kb))
        return out


def set_batched_variant(variant: int, device=None) -> None:
    """Force a batched launch variant (0..7) on the device's context; -1 restores
    the tuned / default choice."""
    dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
    h = _context(dev)
    _check(h, _lib.idcur_id_col_batched_set_variant(h, int(variant)))


def id_col_batched(blocks, **kw) -> list:
    """Column IDs of a list of FP32 blocks in one launch (see :class:`BatchedID`)."""
    plan = BatchedID(blocks, **kw)
    plan.run()
    return plan.results()
