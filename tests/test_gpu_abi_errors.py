"""Argument errors of the C ABI (include/idcur.h): every documented error code
comes back synchronously, with a message, and nothing is enqueued.

A context needs a GPU (idcur_create queries the device), so these run with the
gpu tests; each call is made through the raw ctypes entry points with device
buffers that are valid except for the one argument under test.
"""
import ctypes

import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

import paper_1412_8447_amd as P  # noqa: E402
from paper_1412_8447_amd import _lib, _context  # noqa: E402

F64, F32 = 0, 1
OK, EINVAL, EDTYPE, EWORKSPACE = 0, -1, -2, -3


@pytest.fixture(scope="module")
def env():
    dev = torch.device("cuda", 0)
    h = _context(dev)
    m, n = 64, 48
    A = torch.randn(m, n, dtype=torch.float64, device=dev)
    A32 = A.float()
    bufs = dict(J=torch.zeros(n, dtype=torch.int32, device=dev), I=torch.zeros(m, dtype=torch.int32, device=dev),
                T=torch.zeros(n * n, dtype=torch.float64, device=dev), kout=torch.zeros(2, dtype=torch.int32, device=dev),
                ws=torch.zeros(1 << 24, dtype=torch.uint8, device=dev))
    return h, A, A32, bufs


def _id_col(h, A, o, bufs, *, dtype=None, m=None, n=None, lda=None, ws_bytes=None, J=True, T=True, ldt=None,
            kout=True, Aptr=True):
    mm, nn = A.shape
    dtype = (F64 if A.dtype == torch.float64 else F32) if dtype is None else dtype
    return _lib.idcur_id_col(h, dtype, mm if m is None else m, nn if n is None else n,
                             A.data_ptr() if Aptr else None, nn if lda is None else lda, ctypes.byref(o),
                             bufs["ws"].data_ptr(), bufs["ws"].numel() if ws_bytes is None else ws_bytes,
                             bufs["kout"].data_ptr() if kout else None, bufs["J"].data_ptr() if J else None,
                             bufs["T"].data_ptr() if T else None, nn if ldt is None else ldt)


def _msg(h):
    return _lib.idcur_last_error(h).decode()


def test_valid_call_is_ok(env):
    h, A, _, bufs = env
    assert _id_col(h, A, P.make_opts(5), bufs) == OK
    assert P.sync_status(A.device) == OK


@pytest.mark.parametrize("case", ["m0", "n0", "lda", "k_ge_min", "k_neg", "tol0", "tol_nan", "kmax0", "kmax_big",
                                  "q_neg", "kp_big", "rank_tol", "norms", "sketch_kind", "u_correct", "t_reg",
                                  "null_A", "null_J", "null_T", "null_kout", "ldt", "prec"])
def test_einval(env, case):
    h, A, _, bufs = env
    o = P.make_opts(5)
    kw = {}
    if case == "m0":
        kw["m"] = 0
    elif case == "n0":
        kw["n"] = 0
    elif case == "lda":
        kw["lda"] = A.shape[1] - 1
    elif case == "k_ge_min":
        o = P.make_opts(min(A.shape))
    elif case == "k_neg":
        o = P.make_opts(5)
        o.k = -1
    elif case == "tol0":
        o = P.make_opts(0, tol=0.0, kmax=10)
    elif case == "tol_nan":
        o = P.make_opts(0, tol=float("nan"), kmax=10)
    elif case == "kmax0":
        o = P.make_opts(0, tol=1e-3, kmax=0)
    elif case == "kmax_big":
        o = P.make_opts(0, tol=1e-3, kmax=min(A.shape))
    elif case == "q_neg":
        o = P.make_opts(5, p=4, q=-1)
    elif case == "kp_big":
        o = P.make_opts(5, p=5000)
    elif case == "rank_tol":
        o = P.make_opts(5, rank_tol=-1.0)
    elif case == "norms":
        o.norms = 7
    elif case == "sketch_kind":
        o.sketch = 9
    elif case == "u_correct":
        o.u_correct = 2
    elif case == "t_reg":
        o = P.make_opts(5, t_reg=1.5)
    elif case == "null_A":
        kw["Aptr"] = False
    elif case == "null_J":
        kw["J"] = False
    elif case == "null_T":
        kw["T"] = False
    elif case == "null_kout":
        kw["kout"] = False
    elif case == "ldt":
        kw["ldt"] = A.shape[1] - 6
    elif case == "prec":
        o.prec = 5
    st = _id_col(h, A, o, bufs, **kw)
    assert st == EINVAL, (case, st, _msg(h))
    assert _msg(h), case


def test_edtype(env):
    h, A, A32, bufs = env
    # unknown dtype, and a 16-bit sketch of FP64 data
    assert _id_col(h, A, P.make_opts(5), bufs, dtype=7) == EDTYPE
    assert _id_col(h, A, P.make_opts(5, p=4, prec="bf16"), bufs) == EDTYPE
    assert "FP32" in _msg(h)


def test_eworkspace(env):
    h, A, _, bufs = env
    o = P.make_opts(5, p=4, q=1)
    need = ctypes.c_size_t(0)
    assert _lib.idcur_workspace_bytes(h, 0, F64, A.shape[0], A.shape[1], ctypes.byref(o), ctypes.byref(need)) == OK
    assert need.value > 256
    # the query adds 256 bytes of slack for the caller's alignment; well below
    # the carved size the call refuses
    assert _id_col(h, A, o, bufs, ws_bytes=(need.value - 256) // 2) == EWORKSPACE
    assert "workspace" in _msg(h)
    assert _id_col(h, A, o, bufs, ws_bytes=need.value) == OK
    assert P.sync_status(A.device) == OK


def test_null_context():
    o = P.make_opts(5)
    assert _lib.idcur_id_col(None, F64, 10, 10, None, 10, ctypes.byref(o), None, 0, None, None, None, 10) == EINVAL
