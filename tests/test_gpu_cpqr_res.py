"""GPU parity of the on-chip-slab pivoted QR (Section 2.2, eq. (trunc)): the
FP32 kernel that keeps part of each column group in registers and the rest in
LDS, for matrices of at most 512 rows with too many columns for the register
kernel -- the 500 x 50000 C^T of the rank-500 row ID.

Bars:
* against the register-slab kernel (16 lanes per column) on shapes both cover:
  J, k and T identical. The two run the same arithmetic in the same order; the
  slots the on-chip kernel skips (wholly above the pivot row) would only add
  exact zeros. IDCUR_CPQR_RESCFG=i forces table entry i of the on-chip kernel.
* against the FP64 oracle at full size (500 x 50000): J identical wherever the
  oracle's pivot gap is clear of FP32 noise (1e-4), the ID error within 1.05x
  of the oracle's.
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

# entries of the on-chip kernel's table (cpqr_res_kernel.hpp): (threads, RPL, NC, NL)
RES_CFGS = [(512, 32, 5, 2), (512, 33, 4, 2)]


@contextlib.contextmanager
def res_cfg(i):
    old = os.environ.get("IDCUR_CPQR_RESCFG")
    os.environ["IDCUR_CPQR_RESCFG"] = str(i)
    try:
        yield
    finally:
        if old is None:
            del os.environ["IDCUR_CPQR_RESCFG"]
        else:
            os.environ["IDCUR_CPQR_RESCFG"] = old


def _fp32(m, n, scale, seed):
    return synth.lowrank(m, n, synth.sigma_exp(min(m, n), scale), seed=seed).astype(np.float32)


# shapes the register kernel takes with 16 lanes per column (l <= 256 or
# 500 < l <= 512 rows): ragged tails, a single step, k = l - 1, l not a multiple of 16
@pytest.mark.parametrize("cfg", [0, 1])
@pytest.mark.parametrize("norms", ["downdate", "exact"])
@pytest.mark.parametrize("m,n,k", [(500, 9000, 480), (512, 6001, 511), (200, 3000, 150), (37, 2000, 36),
                                   (129, 3001, 1), (250, 777, 240)])
def test_matches_register_kernel(cfg, norms, m, n, k):
    say(f"on-chip cpqr cfg {cfg} vs register kernel: {m}x{n} k={k} norms={norms}")
    A = _fp32(m, n, max(4.0, m / 8.0), seed=m + 7 * n + k)
    dA = to_dev(A, torch.float32)
    a = P.id_col(dA, k, norms=norms)
    with res_cfg(cfg):
        b = P.id_col(dA, k, norms=norms)
    assert a.k == b.k == k
    check_perm(b.J.cpu().numpy(), n)
    assert torch.equal(a.J, b.J)
    assert torch.equal(a.T, b.T)


@pytest.mark.parametrize("cfg", [1])
@pytest.mark.parametrize("norms", ["downdate", "exact"])
@pytest.mark.parametrize("m,n,k", [(520, 6000, 500), (528, 4001, 527), (513, 3000, 200)])
def test_33_slot_configs_match_register_kernel(cfg, norms, m, n, k):
    """The entries with 33 row slots (sketches of up to 528 rows, such as the
    520 x 20000 sketch of the rank-500 workload) against the register kernel."""
    say(f"on-chip cpqr cfg {cfg} vs register kernel: {m}x{n} k={k} norms={norms}")
    A = _fp32(m, n, 80.0, seed=m + 5 * n + k)
    dA = to_dev(A, torch.float32)
    a = P.id_col(dA, k, norms=norms)
    with res_cfg(cfg):
        b = P.id_col(dA, k, norms=norms)
    assert a.k == b.k == k
    assert torch.equal(a.J, b.J)
    assert torch.equal(a.T, b.T)


@pytest.mark.parametrize("cfg", [0, 1])
def test_rank_deficient(cfg):
    """Exactly rank-r input with k = r + 5: both kernels stop at r, identically."""
    m, n, r = 250, 5000, 61
    say(f"on-chip cpqr cfg {cfg}: rank deficient {m}x{n} r={r}")
    A = synth.lowrank(m, n, np.ones(r), seed=17, rank=r).astype(np.float32)
    dA = to_dev(A, torch.float32)
    a = P.id_col(dA, r + 5)
    with res_cfg(cfg):
        b = P.id_col(dA, r + 5)
    assert a.k == b.k == r
    assert torch.equal(a.J, b.J)
    assert torch.equal(a.T, b.T)


@pytest.mark.parametrize("cfg", [0, 1])
def test_tolerance_mode(cfg):
    """Tolerance mode against the FP64 oracle: the same rank and clear pivots."""
    m, n = 400, 6000
    A = _fp32(m, n, 12.0, seed=23)
    A64 = A.astype(np.float64)
    say(f"on-chip cpqr cfg {cfg}: tolerance mode {m}x{n}")
    ref = oracle.id_col(A64, 300, tol=1e-3)
    with res_cfg(cfg):
        got = P.id_col(to_dev(A, torch.float32), 0, tol=1e-3, kmax=300)
    assert got.k == ref.k
    J = got.J.cpu().numpy()
    check_perm(J, n)
    c = clear_prefix(ref.qr.gaps[: ref.k], 1e-4)
    assert c >= 10
    assert np.array_equal(J[:c], ref.J[:c])
    assert rel_err_id(A64, J, got.T.cpu().numpy()) <= 1.05 * rel_err_id(A64, ref.J, ref.T)


def test_full_size_500x50000_against_oracle():
    """The row ID's shape: 500 x 50000 FP32 (sigma_j = exp(-j/80), as the
    columns of the rank-500 workload's C), the library's own kernel choice;
    k = 450, so that the ID error is a truncation error the two sides can be
    compared on (at k = 500 every ID of a 500-row matrix is exact)."""
    m, n, k = 500, 50000, 450
    say(f"on-chip cpqr at full size {m}x{n} k={k}")
    A = _fp32(m, n, 80.0, seed=1412)
    A64 = A.astype(np.float64)
    got = P.id_col(to_dev(A, torch.float32), k)
    J = got.J.cpu().numpy()
    check_perm(J, n)
    assert got.k == k
    ref = oracle.id_col(A64, k)
    c = clear_prefix(ref.qr.gaps, 1e-4)
    say(f"  clear pivots {c} of {k}")
    assert c >= 20
    assert np.array_equal(J[:c], ref.J[:c])
    e_g, e_o = rel_err_id(A64, J, got.T.cpu().numpy()), rel_err_id(A64, ref.J, ref.T)
    say(f"  e_ID device {e_g:.4e} oracle {e_o:.4e}")
    assert e_g <= 1.05 * e_o


def test_repeat_bitwise():
    """Two calls on the same input give identical J and T."""
    A = _fp32(500, 40000, 80.0, seed=5)
    dA = to_dev(A, torch.float32)
    a = P.id_col(dA, 300)
    b = P.id_col(dA, 300)
    assert torch.equal(a.J, b.J)
    assert torch.equal(a.T, b.T)
