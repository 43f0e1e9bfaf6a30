"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Inputs come from ``synth`` and are handed to both sides. Pivot sets must agree
wherever the oracle's best-vs-runner-up gap is clear of the arithmetic's noise;
T agrees to a tolerance derived from cond(S11) and the dtype; errors agree to a
ratio bound (FP64: 1e-10 relative, FP32: within 1.05x of the oracle)."""
import math

import numpy as np
import pytest

import synth
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

import paper_1412_8447_amd as P  # noqa: E402
from gpu_helpers import say, to_dev, clear_prefix, rel_err_id, check_perm, check_t_fp32  # noqa: E402


def _det_case(m, n, k, seed, decay=8.0):
    return synth.lowrank(m, n, synth.sigma_exp(min(m, n), decay), seed=seed)


# ---------------------------------------------------------------------------
# The Gaussian sketch matrix
# ---------------------------------------------------------------------------
def test_gaussian_matches_oracle_generator():
    say("gaussian 37x1001")
    g = P.gaussian(37, 1001, seed=12345, dtype=torch.float64).cpu().numpy()
    want = oracle.philox.gaussian_omega(37, 1001, seed=12345)
    assert np.abs(g - want).max() <= 1e-12 * max(1.0, np.abs(want).max())
    g32 = P.gaussian(5, 77, seed=(1 << 40) + 3, dtype=torch.float32).cpu().numpy()
    want32 = oracle.philox.gaussian_omega(5, 77, seed=(1 << 40) + 3)
    assert np.abs(g32 - want32).max() <= 1e-6


@pytest.mark.parametrize("m", [400, 402])
def test_sketch_omega_layout(m):
    """The sketch draws Omega^T column-major (coalesced stores when m % 4 == 0):
    the FP64 sketch of the identity is Omega^T exactly, the oracle's Philox draw."""
    k, p, seed = 30, 6, 4321
    say(f"sketch of I_{m}: Omega^T layout")
    Yt = P.sketch(torch.eye(m, dtype=torch.float64, device="cuda"), k, p=p, q=0, seed=seed).cpu().numpy()
    want = oracle.philox.gaussian_omega(k + p, m, seed=seed)
    assert np.abs(Yt - want.T).max() <= 1e-12 * max(1.0, np.abs(want).max())
    assert torch.equal(torch.as_tensor(Yt), P.gaussian(k + p, m, seed=seed, dtype=torch.float64).cpu().T)


# ---------------------------------------------------------------------------
# Deterministic column ID (Algorithm 1)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("m,n,k,norms", [(300, 200, 20, "downdate"), (301, 517, 33, "exact"), (64, 40, 1, "downdate"),
                                         (90, 300, 60, "downdate")])
def test_id_col_det_fp64(m, n, k, norms):
    say(f"id_col det fp64 {m}x{n} k={k} norms={norms}")
    A = _det_case(m, n, k, seed=m + n + k)
    ref = oracle.id_col(A, k)
    got = P.id_col(to_dev(A, torch.float64), k, norms=norms)
    J = got.J.cpu().numpy()
    check_perm(J, n)
    assert got.k == k
    c = clear_prefix(ref.qr.gaps, 1e-10)
    assert c == k, "test input should have clear gaps"
    assert np.array_equal(J[:k], ref.J[:k])
    assert np.array_equal(J[k:], ref.J[k:])
    T = got.T.cpu().numpy()
    scale = max(1.0, np.abs(ref.T).max())
    assert np.abs(T - ref.T).max() <= 1e-9 * scale
    e_g, e_o = rel_err_id(A, J, T), rel_err_id(A, ref.J, ref.T)
    assert abs(e_g / e_o - 1) <= 1e-10


@pytest.mark.parametrize("m,n,k", [(500, 300, 25), (257, 700, 40)])
def test_id_col_det_fp32(m, n, k):
    say(f"id_col det fp32 {m}x{n} k={k}")
    A = _det_case(m, n, k, seed=7 * m + n).astype(np.float32)
    ref = oracle.id_col(A.astype(np.float64), k)
    got = P.id_col(to_dev(A, torch.float32), k)
    J = got.J.cpu().numpy()
    check_perm(J, n)
    c = clear_prefix(ref.qr.gaps, 1e-4)
    assert c >= min(k, 10)
    assert np.array_equal(J[:c], ref.J[:c])
    # T element-wise: Y = A itself in the deterministic ID
    check_t_fp32(A, J, k, got.T.cpu().numpy(), "det fp32")
    e_g, e_o = rel_err_id(A.astype(np.float64), J, got.T.cpu().numpy()), rel_err_id(A.astype(np.float64), ref.J, ref.T)
    assert e_g <= 1.05 * e_o


def test_id_col_det_fp64_full_config():
    """2000 x 1000, sigma_j = exp(-j/10), k = 50 (the deterministic FP64 workload)."""
    cfg = synth.CONFIGS["det_fp64_2000x1000_k50"]
    say("id_col det fp64 full 2000x1000 k=50")
    A = synth.lowrank(cfg.m, cfg.n, cfg.spectrum(), seed=2024)
    ref = oracle.id_col(A, cfg.k)
    for norms in ("downdate", "exact"):
        got = P.id_col(to_dev(A, torch.float64), cfg.k, norms=norms)
        J = got.J.cpu().numpy()
        assert np.array_equal(J, ref.J)
        T = got.T.cpu().numpy()
        assert np.linalg.norm(T - ref.T) <= 1e-10 * np.linalg.norm(ref.T)
        e_g, e_o = rel_err_id(A, J, T), rel_err_id(A, ref.J, ref.T)
        assert abs(e_g / e_o - 1) <= 1e-10
        assert e_o >= cfg.frobenius_floor()


# ---------------------------------------------------------------------------
# Randomized column ID with a caller-supplied Omega (Algorithm 4 + power steps)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("dtype,q", [(torch.float64, 0), (torch.float64, 1), (torch.float32, 1)])
def test_id_col_sketched_matches_oracle(dtype, q):
    m, n, k, p = 700, 450, 30, 10
    say(f"id_col sketch {dtype} q={q} {m}x{n} k={k} p={p}")
    A = synth.lowrank(m, n, synth.sigma_exp(min(m, n), 6.0), seed=99)
    om = synth.gaussian(k + p, m, seed=5)
    npdt = np.float64 if dtype == torch.float64 else np.float32
    A_in, om_in = A.astype(npdt), om.astype(npdt)
    ref = oracle.id_col(A_in.astype(np.float64), k, omega=om_in.astype(np.float64), q=q)
    got = P.id_col(to_dev(A_in, dtype), k, p=p, q=q, omega=to_dev(om_in, dtype))
    J = got.J.cpu().numpy()
    check_perm(J, n)
    thr = 1e-9 if dtype == torch.float64 else 1e-4
    c = clear_prefix(ref.qr.gaps, thr)
    assert c >= 5
    assert np.array_equal(J[:c], ref.J[:c])
    A64 = A_in.astype(np.float64)
    e_g, e_o = rel_err_id(A64, J, got.T.cpu().numpy()), rel_err_id(A64, ref.J, ref.T)
    if dtype == torch.float64 and c == k:
        assert abs(e_g / e_o - 1) <= 1e-8
        assert np.abs(got.T.cpu().numpy() - ref.T).max() <= 1e-8 * max(1.0, np.abs(ref.T).max())
    if dtype == torch.float32:
        # T of the device's skeleton on the oracle's sketch of the same inputs
        check_t_fp32(ref.Y, J, k, got.T.cpu().numpy(), f"sketch fp32 q={q}")
    assert e_g <= 1.05 * e_o


def test_id_col_device_generated_omega():
    """Omega drawn on the device from the seed equals the oracle's Philox draw."""
    m, n, k, p = 400, 300, 20, 10
    say("id_col device omega")
    A = synth.lowrank(m, n, synth.sigma_exp(min(m, n), 5.0), seed=17)
    om = oracle.philox.gaussian_omega(k + p, m, seed=777)
    ref = oracle.id_col(A, k, omega=om, q=1)
    got = P.id_col(to_dev(A, torch.float64), k, p=p, q=1, seed=777)
    J = got.J.cpu().numpy()
    c = clear_prefix(ref.qr.gaps, 1e-9)
    assert np.array_equal(J[:c], ref.J[:c])
    assert rel_err_id(A, J, got.T.cpu().numpy()) <= 1.05 * rel_err_id(A, ref.J, ref.T)


# ---------------------------------------------------------------------------
# Row ID, two-sided ID, CUR
# ---------------------------------------------------------------------------
def test_id_row_det_fp64():
    m, n, k = 250, 400, 30
    say(f"id_row {m}x{n}")
    A = _det_case(m, n, k, seed=3)
    ref = oracle.id_row(A, k)
    got = P.id_row(to_dev(A, torch.float64), k)
    I = got.J.cpu().numpy()
    check_perm(I, m)
    assert np.array_equal(I, ref.J)
    assert np.abs(got.T.cpu().numpy() - ref.T).max() <= 1e-9 * max(1.0, np.abs(ref.T).max())


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_two_sided_and_cur_det(dtype):
    m, n, k = 420, 310, 24
    say(f"two-sided / cur det {dtype} {m}x{n} k={k}")
    A = _det_case(m, n, k, seed=11, decay=6.0)
    npdt = np.float64 if dtype == torch.float64 else np.float32
    A_in = A.astype(npdt)
    A64 = A_in.astype(np.float64)
    ref = oracle.cur(A64, k)
    ts = P.id_two_sided(to_dev(A_in, dtype), k)
    assert ts.k == k and ts.k_row == k
    J, I = ts.J.cpu().numpy(), ts.I.cpu().numpy()
    check_perm(J, n)
    check_perm(I, m)
    cref = clear_prefix(ref.ts.col.qr.gaps, 1e-9 if dtype == torch.float64 else 1e-4)
    assert np.array_equal(J[:cref], ref.ts.col.J[:cref])
    # two-sided error equals the column-ID error (no extra error, Section 2.4)
    if dtype == torch.float32:
        # T and Tr element-wise: the column ID is of A itself, the row ID of C^T
        check_t_fp32(A64, J, k, ts.T.cpu().numpy(), "two-sided T")
        check_t_fp32(A64[:, J[:k]].T, I, k, ts.Tr.cpu().numpy(), "two-sided Tr")
    e2 = oracle.e_two_sided(A64, J, ts.T.cpu().numpy(), I, ts.Tr.cpu().numpy())
    e1 = oracle.e_id(A64, J, ts.T.cpu().numpy())
    tol = 1e-9 if dtype == torch.float64 else 2e-3
    assert abs(e2 / e1 - 1) <= tol
    # row ID of C is exact up to rounding
    C = A64[:, J[:k]]
    W = oracle.w_from(I, ts.Tr.cpu().numpy().astype(np.float64), m)
    rel = np.linalg.norm(C - W @ C[I[:k]]) / np.linalg.norm(C)
    assert rel <= (1e-12 if dtype == torch.float64 else 1e-5)
    cu = P.cur(to_dev(A_in, dtype), k)
    assert cu.k == k and cu.k_row == k
    Cg, Ug, Rg = (x.cpu().numpy().astype(np.float64) for x in (cu.C, cu.U, cu.R))
    assert np.array_equal(Cg, A64[:, cu.J.cpu().numpy()[:k]])
    assert np.array_equal(Rg, A64[cu.I.cpu().numpy()[:k]])
    e_g = oracle.e_cur(A64, Cg, Ug, Rg)
    e_o = oracle.e_cur(A64, ref.C, ref.U, ref.R)
    if dtype == torch.float64:
        assert abs(e_g / e_o - 1) <= 1e-8
        assert np.abs(Ug - ref.U).max() <= 1e-7 * np.abs(ref.U).max()
    else:
        assert e_g <= 1.05 * e_o


# ---------------------------------------------------------------------------
# Degenerate cases
# ---------------------------------------------------------------------------
def test_exact_rank_deficiency_fp64():
    m, n, r = 200, 150, 7
    say("rank deficiency")
    A = synth.lowrank(m, n, synth.sigma_pow(r, 1.0), seed=31, rank=r)
    got = P.id_col(to_dev(A, torch.float64), r + 5)
    assert got.k == r
    e = rel_err_id(A, got.J.cpu().numpy(), got.T.cpu().numpy())
    assert e <= 1e-12
    cu = P.cur(to_dev(A, torch.float64), r)
    e_c = oracle.e_cur(A, *(x.cpu().numpy() for x in (cu.C, cu.U, cu.R)))
    assert e_c <= 1e-11


def test_tolerance_mode_fp64():
    m, n = 300, 260
    say("tolerance mode")
    A = synth.lowrank(m, n, synth.sigma_exp(min(m, n), 5.0), seed=41)
    tol = 1e-4
    ref = oracle.id_col(A, 200, tol=tol)
    got = P.id_col(to_dev(A, torch.float64), 0, tol=tol, kmax=200)
    assert got.k == ref.k
    assert np.array_equal(got.J.cpu().numpy(), ref.J)
    assert rel_err_id(A, got.J.cpu().numpy(), got.T.cpu().numpy()) <= tol * (1 + 1e-9)


def test_ties_smallest_index():
    Y = np.zeros((6, 9))
    Y[0, 0], Y[1, 5], Y[2, 2], Y[3, 7], Y[4, 8] = 1.0, 2.0, 2.0, 0.5, 2.0
    say("ties")
    got = P.id_col(to_dev(Y, torch.float64), 3)
    assert list(got.J.cpu().numpy()[:3]) == [2, 5, 8]


# ---------------------------------------------------------------------------
# Error measurement kernels
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_error_kernels_match_oracle(dtype):
    m, n, k = 333, 517, 21
    say(f"error kernels {dtype}")
    npdt = np.float64 if dtype == torch.float64 else np.float32
    A = synth.lowrank(m, n, synth.sigma_exp(min(m, n), 7.0), seed=51).astype(npdt)
    A64 = A.astype(np.float64)
    dA = to_dev(A, dtype)
    ci = P.id_col(dA, k)
    e2 = P.id_error(dA, ci.J, ci.T, ci.kout, k).cpu().numpy()
    want = oracle.e_id(A64, ci.J.cpu().numpy(), ci.T.cpu().numpy().astype(np.float64))
    assert abs(math.sqrt(e2[0] / e2[1]) / want - 1) <= 1e-9
    assert abs(e2[1] / (A64 ** 2).sum() - 1) <= 1e-12
    cu = P.cur(dA, k)
    e3 = P.cur_error(dA, cu.C, cu.U, cu.R, cu.kout, k).cpu().numpy()
    want3 = oracle.e_cur(A64, *(x.cpu().numpy().astype(np.float64) for x in (cu.C, cu.U, cu.R)))
    assert abs(math.sqrt(e3[0] / e3[1]) / want3 - 1) <= 1e-9
