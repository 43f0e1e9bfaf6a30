"""GPU parity of the truncated-SVD interpolation matrix (Section 4.1: the
stabilized pseudo-inverse of S11 in eq. (lsqr_for_T), opts t_svd) against the
FP64 oracle.

The threshold is placed between two singular values of S11 (from the oracle's
factor), so that both sides drop the same terms. Bars: FP64 -- J identical, T
within 1e-8 relative Frobenius (the Jacobi SVD and the oracle's LAPACK SVD agree
to about cond(S11 kept) u); FP32 -- J on the clear prefix, T against the FP64
truncated least squares of the device's skeleton on the oracle's sketch within
max(1e-3, 50 cond u32), the error within 1.05x of the oracle's.
"""
import numpy as np
import pytest

import synth
import oracle

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skip(reason="the truncated-SVD path is switched off: the GPU run that first included it "
                                      "ended with a device fault whose cause has not been shown (the library "
                                      "rejects t_svd > 0 with IDCUR_EINVAL)")]

if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

import paper_1412_8447_amd as P  # noqa: E402
from gpu_helpers import say, to_dev, clear_prefix, rel_err_id, check_perm  # noqa: E402

U32 = 2.0 ** -24


def _cut(S11, i):
    """A relative threshold strictly between singular values i - 1 and i."""
    s = np.linalg.svd(S11, compute_uv=False)
    return float(np.sqrt(s[i] * s[i - 1]) / s[0]), s


@pytest.mark.parametrize("m,n,k,decay,drop", [(600, 400, 40, 3.0, 6), (300, 900, 64, 4.0, 10), (257, 130, 33, 2.5, 1)])
def test_tsvd_det_fp64(m, n, k, decay, drop):
    """Deterministic ID (Y = A) in FP64 with the last `drop` singular directions
    of S11 cut."""
    say(f"tsvd det fp64 {m}x{n} k={k} drop={drop}")
    A = synth.lowrank(m, n, synth.sigma_exp(min(m, n), decay), seed=m + n + k)
    plain = oracle.id_col(A, k)
    assert clear_prefix(plain.qr.gaps, 1e-10) == k
    thr, s = _cut(plain.qr.S[:k, :k], k - drop)
    say(f"  cond(S11) {s[0] / s[-1]:.3e}, threshold {thr:.3e}")
    ref = oracle.id_col(A, k, t_svd=thr)
    got = P.id_col(to_dev(A, torch.float64), k, t_svd=thr)
    J = got.J.cpu().numpy()
    check_perm(J, n)
    assert np.array_equal(J, ref.J)
    T = got.T.cpu().numpy()
    dT = np.linalg.norm(T - ref.T) / np.linalg.norm(ref.T)
    say(f"  |dT|/|T| = {dT:.3e}")
    assert dT <= 1e-8
    e_g, e_o = rel_err_id(A, J, T), rel_err_id(A, ref.J, ref.T)
    assert abs(e_g / e_o - 1) <= 1e-8
    # the cut changed T: it differs from the plain interpolation matrix
    assert np.linalg.norm(ref.T - plain.T) > 1e-6 * np.linalg.norm(plain.T)


def test_tsvd_tiny_threshold_is_plain_t():
    """Nothing dropped: the Jacobi route gives the plain T = S11^{-1} S12."""
    m, n, k = 500, 300, 30
    A = synth.lowrank(m, n, synth.sigma_exp(min(m, n), 8.0), seed=9)
    say("tsvd tiny threshold fp64")
    plain = P.id_col(to_dev(A, torch.float64), k)
    stab = P.id_col(to_dev(A, torch.float64), k, t_svd=1e-15)
    assert torch.equal(plain.J, stab.J)
    Tp, Ts = plain.T.cpu().numpy(), stab.T.cpu().numpy()
    assert np.linalg.norm(Ts - Tp) <= 1e-9 * np.linalg.norm(Tp)


def test_tsvd_tolerance_mode_fp64():
    """Tolerance mode: the rank k_out < kmax comes from the device; the Jacobi
    SVD and the scaling act on the leading k_out x k_out block only."""
    m, n = 400, 500
    A = synth.lowrank(m, n, synth.sigma_exp(min(m, n), 5.0), seed=21)
    say("tsvd tolerance mode fp64")
    ref0 = oracle.id_col(A, 120, tol=1e-5)
    kk = ref0.k
    thr, _ = _cut(ref0.qr.S[:kk, :kk], kk - 4)
    ref = oracle.id_col(A, 120, tol=1e-5, t_svd=thr)
    got = P.id_col(to_dev(A, torch.float64), 0, tol=1e-5, kmax=120, t_svd=thr)
    assert got.k == ref.k
    J = got.J.cpu().numpy()
    assert np.array_equal(J[: got.k], ref.J[: ref.k])
    T = got.T.cpu().numpy()
    assert np.linalg.norm(T - ref.T) <= 1e-8 * np.linalg.norm(ref.T)


def test_tsvd_sketched_fp32():
    """Randomized FP32 ID (Algorithm 4, q = 1) with the caller's Omega."""
    m, n, k, p = 3000, 2000, 60, 10
    say(f"tsvd sketched fp32 {m}x{n} k={k}")
    A = synth.lowrank(m, n, synth.sigma_exp(min(m, n), 10.0), seed=31).astype(np.float32)
    om = synth.gaussian(k + p, m, seed=32).astype(np.float32)
    A64, om64 = A.astype(np.float64), om.astype(np.float64)
    plain = oracle.id_col(A64, k, omega=om64, q=1)
    thr, s = _cut(plain.qr.S[:k, :k], k - 5)
    ref = oracle.id_col(A64, k, omega=om64, q=1, t_svd=thr)
    got = P.id_col(to_dev(A, torch.float32), k, p=p, q=1, omega=to_dev(om, torch.float32), t_svd=thr)
    J = got.J.cpu().numpy()
    check_perm(J, n)
    c = clear_prefix(ref.qr.gaps, 1e-4)
    assert c >= 10
    assert np.array_equal(J[:c], ref.J[:c])
    T = got.T.cpu().numpy().astype(np.float64)
    # the truncated least squares of the device skeleton on the oracle's sketch:
    # S11 = Q1^T Y1, so the truncated pseudo-inverse of S11 applied to Q1^T Y2 is
    # that of Y1 applied to Y2 (LAPACK gelsd with rcond = thr)
    Y = ref.Y
    T_ref = np.linalg.lstsq(Y[:, J[:k]], Y[:, J[k:]], rcond=thr)[0]
    sk = np.linalg.svd(Y[:, J[:k]], compute_uv=False)
    kept = sk[sk >= thr * sk[0]]
    cond = kept[0] / kept[-1]
    dT = np.linalg.norm(T - T_ref) / np.linalg.norm(T_ref)
    bound = max(1e-3, 50.0 * cond * U32)
    say(f"  |dT|/|T| = {dT:.3e} (cond of the kept part {cond:.3e}, bound {bound:.3e})")
    assert dT <= bound
    assert rel_err_id(A64, J, T) <= 1.05 * rel_err_id(A64, ref.J, ref.T)


def test_tsvd_cur_fp64():
    """CUR (Algorithm 3) with both interpolation matrices truncated."""
    m, n, k = 700, 500, 30
    A = synth.lowrank(m, n, synth.sigma_exp(min(m, n), 4.0), seed=41)
    plain = oracle.cur(A, k)
    thr, _ = _cut(plain.ts.col.qr.S[:k, :k], k - 3)
    say(f"tsvd cur fp64 threshold {thr:.3e}")
    ref = oracle.cur(A, k, t_svd=thr)
    got = P.cur(to_dev(A, torch.float64), k, t_svd=thr)
    assert np.array_equal(got.J.cpu().numpy()[:k], ref.ts.col.J[:k])
    Cg, Ug, Rg = (x.cpu().numpy() for x in (got.C, got.U, got.R))
    e_g = oracle.e_cur(A, Cg, Ug, Rg)
    e_o = oracle.e_cur(A, ref.C, ref.U, ref.R)
    say(f"  CUR error device {e_g:.4e} oracle {e_o:.4e}")
    assert abs(e_g / e_o - 1) <= 1e-6
