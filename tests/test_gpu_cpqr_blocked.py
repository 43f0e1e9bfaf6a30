"""GPU parity of the blocked pivoted QR (panels of reflectors, trailing update
on the matrix cores; Section 2.2, eq. (trunc)) against the FP64 oracle.

The kernel serves the shapes whose columns do not fit in registers: the
deterministic comparator (Y = A, thousands of rows: the tall form, rows split
over the workgroups) and short, very wide matrices such as the C^T of a
rank-500 CUR (the short form, reflectors in LDS). IDCUR_CPQR_SLAB forces a
kernel for a test: 1 the blocked kernel's own choice, 2 its tall form, 3 the
unblocked slab kernel.

Bars: FP64 -- J identical wherever the oracle's pivot gap is clear (1e-10), T
within 1e-10 relative Frobenius, error ratio within 1e-10; FP32 -- J identical
on the clear prefix (gap 1e-4), the ID error within 1.05x of the oracle's.
"""
import contextlib
import os

import numpy as np
import pytest

import synth
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

import paper_1412_8447_amd as P  # noqa: E402
from gpu_helpers import say, to_dev, clear_prefix, rel_err_id, check_perm  # noqa: E402


@contextlib.contextmanager
def kernel(which):
    old = os.environ.get("IDCUR_CPQR_SLAB")
    os.environ["IDCUR_CPQR_SLAB"] = which
    try:
        yield
    finally:
        if old is None:
            del os.environ["IDCUR_CPQR_SLAB"]
        else:
            os.environ["IDCUR_CPQR_SLAB"] = old


def _check_fp64(A, k, got, ref):
    n = A.shape[1]
    J = got.J.cpu().numpy()
    check_perm(J, n)
    assert got.k == k
    c = clear_prefix(ref.qr.gaps, 1e-10)
    assert c == k, "test input should have clear gaps"
    assert np.array_equal(J, ref.J)
    T = got.T.cpu().numpy()
    assert np.linalg.norm(T - ref.T) <= 1e-10 * max(1.0, np.linalg.norm(ref.T))
    e_g, e_o = rel_err_id(A, J, T), rel_err_id(A, ref.J, ref.T)
    assert abs(e_g / e_o - 1) <= 1e-10


@pytest.mark.parametrize("which", ["1", "2", "3"])
@pytest.mark.parametrize("norms", ["downdate", "exact"])
def test_det_fp64_full_config(which, norms):
    """2000 x 1000, sigma_j = exp(-j/10), k = 50, every slab kernel."""
    cfg = synth.CONFIGS["det_fp64_2000x1000_k50"]
    say(f"blocked cpqr: det fp64 2000x1000 k=50 kernel={which} norms={norms}")
    A = synth.lowrank(cfg.m, cfg.n, cfg.spectrum(), seed=2024)
    ref = oracle.id_col(A, cfg.k)
    with kernel(which):
        got = P.id_col(to_dev(A, torch.float64), cfg.k, norms=norms)
    _check_fp64(A, cfg.k, got, ref)


# ragged shapes: panels crossed (k > 32), l below the grid size (tall form with
# empty row ranges), few columns per workgroup, a single step
@pytest.mark.parametrize("which", ["1", "2"])
@pytest.mark.parametrize("m,n,k", [(301, 517, 45), (90, 300, 60), (1000, 37, 36), (70, 3000, 69), (64, 40, 1),
                                   (600, 2100, 130)])
def test_det_fp64_ragged(which, m, n, k):
    say(f"blocked cpqr: det fp64 {m}x{n} k={k} kernel={which}")
    A = synth.lowrank(m, n, synth.sigma_exp(min(m, n), max(4.0, k / 5.0)), seed=m + 3 * n + k)
    ref = oracle.id_col(A, k)
    with kernel(which):
        got = P.id_col(to_dev(A, torch.float64), k)
    _check_fp64(A, k, got, ref)


@pytest.mark.parametrize("which", ["1", "2"])
def test_det_fp64_rank_deficient(which):
    """Exactly rank-r input with k = r + 3: k_out = r and exact reconstruction."""
    m, n, r = 400, 700, 37
    say(f"blocked cpqr: rank deficient fp64 {m}x{n} r={r} kernel={which}")
    A = synth.lowrank(m, n, np.ones(r), seed=11, rank=r)
    with kernel(which):
        got = P.id_col(to_dev(A, torch.float64), r + 3)
    assert got.k == r
    J = got.J.cpu().numpy()
    check_perm(J, n)
    assert rel_err_id(A, J, got.T.cpu().numpy()) <= 1e-12


@pytest.mark.parametrize("which", ["1", "2"])
def test_tolerance_mode_fp64(which):
    m, n = 500, 800
    A = synth.lowrank(m, n, synth.sigma_exp(min(m, n), 9.0), seed=5)
    say(f"blocked cpqr: tolerance mode fp64 kernel={which}")
    ref = oracle.id_col(A, 200, tol=1e-6)
    with kernel(which):
        got = P.id_col(to_dev(A, torch.float64), 0, tol=1e-6, kmax=200)
    assert got.k == ref.k
    J = got.J.cpu().numpy()
    assert np.array_equal(J[: got.k], ref.J[: ref.k])
    assert rel_err_id(A, J, got.T.cpu().numpy()) <= 1e-6


@pytest.mark.parametrize("which", ["1", "2"])
def test_det_fp32_tall(which):
    """FP32, Y = A with 4000 rows: the comparator's shape class."""
    m, n, k = 4000, 1500, 100
    say(f"blocked cpqr: det fp32 {m}x{n} k={k} kernel={which}")
    A = synth.lowrank(m, n, synth.sigma_pow(min(m, n), 2.0), seed=31).astype(np.float32)
    A64 = A.astype(np.float64)
    ref = oracle.id_col(A64, k)
    with kernel(which):
        got = P.id_col(to_dev(A, torch.float32), k)
    J = got.J.cpu().numpy()
    check_perm(J, n)
    c = clear_prefix(ref.qr.gaps, 1e-4)
    assert c >= 10
    assert np.array_equal(J[:c], ref.J[:c])
    T = got.T.cpu().numpy()
    if np.array_equal(J[:k], ref.J[:k]):
        assert np.linalg.norm(T - ref.T) <= 1e-3 * np.linalg.norm(ref.T)
    assert rel_err_id(A64, J, T) <= 1.05 * rel_err_id(A64, ref.J, ref.T)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_short_form_wide(dtype):
    """A 300 x 30000 matrix, k = 250 (deterministic): too many columns per CU
    for the register kernel, the short form of the blocked kernel (forced: FP32
    slabs of this size otherwise go to the on-chip-slab kernel)."""
    m, n, k = 300, 30000, 250
    say(f"blocked cpqr: short-wide det {dtype} {m}x{n} k={k}")
    A = synth.lowrank(m, n, synth.sigma_exp(m, 60.0), seed=77)
    npdt = np.float32 if dtype == torch.float32 else np.float64
    A_in = A.astype(npdt)
    A64 = A_in.astype(np.float64)
    ref = oracle.id_col(A64, k)
    with kernel("1"):
        got = P.id_col(to_dev(A_in, dtype), k)
    J = got.J.cpu().numpy()
    check_perm(J, n)
    thr = 1e-4 if dtype == torch.float32 else 1e-10
    c = clear_prefix(ref.qr.gaps, thr)
    say(f"  clear pivots {c} of {k}")
    assert c >= (5 if dtype == torch.float32 else k)
    assert np.array_equal(J[:c], ref.J[:c])
    T = got.T.cpu().numpy()
    e_g, e_o = rel_err_id(A64, J, T), rel_err_id(A64, ref.J, ref.T)
    say(f"  e_ID device {e_g:.4e} oracle {e_o:.4e}")
    if dtype == torch.float64 and c == k:
        assert np.linalg.norm(T - ref.T) <= 1e-9 * np.linalg.norm(ref.T)
        assert abs(e_g / e_o - 1) <= 1e-9
    assert e_g <= 1.05 * e_o


def test_blocked_deterministic_repeat():
    """Two calls on the same input give bitwise identical J and T (tall form)."""
    m, n, k = 3000, 900, 70
    A = synth.lowrank(m, n, synth.sigma_pow(min(m, n), 2.0), seed=3).astype(np.float32)
    dA = to_dev(A, torch.float32)
    with kernel("2"):
        a = P.id_col(dA, k)
        b = P.id_col(dA, k)
    assert torch.equal(a.J, b.J)
    assert torch.equal(a.T, b.T)
