"""idcur_id_col_noalloc (the column ID without a workspace, for callers that
cannot allocate) against idcur_id_col on the same inputs: identical J, T and
k_out, on two calls in a row, the second with a smaller input, plus the
size check that rejects problems above the fixed scratch array."""
import ctypes

import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

import paper_1412_8447_amd as P  # noqa: E402
from gpu_helpers import say, to_dev  # noqa: E402

SCRATCH = 64 << 20


def _ws(A, o):
    h = P._context(A.device)
    nb = ctypes.c_size_t(0)
    code = 0 if A.dtype == torch.float64 else 1
    assert P._lib.idcur_workspace_bytes(h, P.OP_ID_COL, code, A.shape[0], A.shape[1], ctypes.byref(o),
                                        ctypes.byref(nb)) == 0
    return nb.value


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_noalloc_matches_id_col_twice(dtype):
    npdt = np.float32 if dtype == torch.float32 else np.float64
    cases = [(2400, 1600, 100, 10, 1), (900, 700, 40, 8, 0)]   # the second call is smaller
    for (m, n, k, p, q) in cases:
        A = to_dev(synth.lowrank(m, n, synth.sigma_pow(min(m, n), 2.0), seed=m + n).astype(npdt), dtype)
        o = P.make_opts(k, p=p, q=q, seed=5)
        need = _ws(A, o)
        say(f"noalloc {dtype} {m}x{n} k={k} p={p} q={q}: workspace {need} bytes")
        assert need <= SCRATCH
        ref = P.id_col(A, k, p=p, q=q, seed=5)
        got = P.id_col_noalloc(A, k, p=p, q=q, seed=5)
        assert got.k == ref.k == k
        assert torch.equal(got.J, ref.J)
        assert torch.equal(got.T, ref.T)


def test_noalloc_tolerance_mode_and_rank_deficiency():
    m, n, r = 500, 400, 23
    A = to_dev(synth.lowrank(m, n, np.ones(r), seed=3, rank=r), torch.float64)
    ref = P.id_col(A, r + 6)
    got = P.id_col_noalloc(A, r + 6)
    assert got.k == ref.k == r
    assert torch.equal(got.J, ref.J) and torch.equal(got.T, ref.T)
    B = to_dev(synth.lowrank(m, n, synth.sigma_exp(min(m, n), 6.0), seed=4), torch.float64)
    ref = P.id_col(B, 0, tol=1e-5, kmax=100)
    got = P.id_col_noalloc(B, 0, tol=1e-5, kmax=100)
    assert got.k == ref.k
    assert torch.equal(got.J, ref.J) and torch.equal(got.T, ref.T)


def test_noalloc_workspace_of_the_fp32_workload():
    """For the record: the workspace the FP32 20000 x 10000, k = 200 column ID
    needs, and whether it fits the fixed scratch array."""
    A = torch.zeros(20000, 10000, dtype=torch.float32, device="cuda")
    need = _ws(A, P.make_opts(200, p=10, q=1, seed=1))
    say(f"noalloc: FP32 20000x10000 k=200 p=10 q=1 needs {need} bytes ({'fits' if need <= SCRATCH else 'too large'})")


def test_noalloc_rejects_problems_above_the_scratch():
    m, n, k = 20000, 10000, 200
    A = torch.zeros(m, n, dtype=torch.float32, device="cuda")
    o = P.make_opts(k, p=1000, q=2, seed=1)
    need = _ws(A, o)
    say(f"noalloc size check: {need} bytes needed")
    assert need > SCRATCH
    with pytest.raises(P.IDCurError) as ei:
        P.id_col_noalloc(A, k, p=1000, q=2, seed=1)
    assert ei.value.code == -3
    assert "64" in str(ei.value) or "bytes" in str(ei.value)
