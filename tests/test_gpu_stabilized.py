"""GPU parity of the Tikhonov-stabilized interpolation matrices (Section 4.1,
eq. (lsqr_for_T) with a regularization term; opts t_reg) against the FP64
oracle: same pivots on clear gaps, T within tolerance, the norm bound
|T|_2 <= |S12|_2 / (2 lam) at every size, and the approximation error at the
full 20000 x 10000 workload."""
import numpy as np
import pytest

import synth
import oracle
import oracle.decomp as D
from oracle.stabilized import interp_tikhonov, tikhonov_weight

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

import paper_1412_8447_amd as P  # noqa: E402
from gpu_helpers import say, to_dev, clear_prefix, check_perm  # noqa: E402


@pytest.mark.parametrize("m,n,k,delta", [(300, 200, 40, 1e-6), (257, 333, 37, 1e-4), (129, 70, 64, 1e-2)])
def test_col_id_fp64(m, n, k, delta):
    """Graded singular values (cond(S11) up to ~1e13): pivots identical, T within
    1e-8 of the oracle's (relative to its largest entry)."""
    say(f"stabilized T fp64 {m}x{n} k={k} t_reg={delta}")
    A = synth.lowrank(m, n, synth.sigma_exp(min(m, n), 2.5), seed=400 + k)
    ref = D.id_col(A, k, t_reg=delta)
    got = P.id_col(to_dev(A, torch.float64), k, t_reg=delta)
    assert got.k == ref.k == k
    assert np.array_equal(got.J.cpu().numpy(), ref.J)
    T = got.T.cpu().numpy()
    err = np.abs(T - ref.T).max() / max(1.0, np.abs(ref.T).max())
    say(f"  max |T - T_oracle| / max(1, |T|) = {err:.3e}")
    assert err <= 1e-8
    # the norm bound of the Tikhonov solution
    S = ref.qr.S
    lam = tikhonov_weight(S[:, :k], delta)
    assert np.linalg.norm(T, 2) <= np.linalg.norm(S[:, k:], 2) / (2 * lam) * (1 + 1e-6)


def test_col_id_fp32():
    m, n, k, delta = 400, 300, 30, 1e-3
    say(f"stabilized T fp32 {m}x{n} k={k} t_reg={delta}")
    A = synth.lowrank(m, n, synth.sigma_exp(min(m, n), 4.0), seed=410).astype(np.float32)
    ref = D.id_col(A.astype(np.float64), k, t_reg=delta)
    got = P.id_col(to_dev(A, torch.float32), k, t_reg=delta)
    assert np.array_equal(got.J.cpu().numpy()[:k], ref.J[:k])
    T = got.T.cpu().numpy().astype(np.float64)
    err = np.abs(T - ref.T).max() / max(1.0, np.abs(ref.T).max())
    say(f"  max |T - T_oracle| / max(1, |T|) = {err:.3e}")
    assert err <= 1e-3


def test_two_sided_fp64_both_matrices():
    """t_reg applies to the column T and to the row ID's Tr of a two-sided ID."""
    m, n, k, delta = 280, 220, 24, 1e-5
    say(f"stabilized two-sided fp64 {m}x{n} k={k}")
    A = synth.lowrank(m, n, synth.sigma_exp(min(m, n), 3.0), seed=420)
    ref = D.two_sided(A, k, t_reg=delta)
    got = P.id_two_sided(to_dev(A, torch.float64), k, t_reg=delta)
    assert np.array_equal(got.J.cpu().numpy(), ref.col.J)
    assert np.array_equal(got.I.cpu().numpy(), ref.row.J)
    for g, r in ((got.T, ref.col.T), (got.Tr, ref.row.T)):
        g = g.cpu().numpy()
        assert np.abs(g - r).max() <= 1e-8 * max(1.0, np.abs(r).max())


def test_zero_weight_is_the_plain_solve():
    """A tiny weight on a well-conditioned problem gives the back-substitution's T."""
    m, n, k = 200, 150, 20
    A = synth.lowrank(m, n, synth.sigma_exp(min(m, n), 30.0), seed=430)
    Ad = to_dev(A, torch.float64)
    a = P.id_col(Ad, k).T.cpu().numpy()
    b = P.id_col(Ad, k, t_reg=1e-9).T.cpu().numpy()
    assert np.abs(a - b).max() <= 1e-9 * max(1.0, np.abs(a).max())


@pytest.mark.parametrize("bad", [-1e-3, 1.0, 2.0, float("nan")])
def test_bad_weight_rejected(bad):
    A = torch.zeros(20, 10, dtype=torch.float64, device="cuda")
    with pytest.raises(P.IDCurError):
        P.id_col(A, 3, t_reg=bad)


def test_full_size_fp32_sketched():
    """FP32 20000 x 10000, sigma_j = (j+1)^-2, k = 200, p = 10, q = 1, t_reg =
    1e-4: the ID error within 1.02x of the unregularized ID's (same sketch,
    same pivots) and T within the norm bound of the GPU's own S12 scale."""
    m, n, k = 20000, 10000, 200
    say(f"stabilized T full size fp32 {m}x{n} k={k}")
    sig = (np.arange(min(m, n), dtype=np.float64) + 1.0) ** -2.0
    A = synth.lowrank_torch(m, n, sig, seed=440, device="cuda").to(torch.float32).contiguous()
    kw = dict(p=10, q=1, seed=5)
    a = P.id_col(A, k, **kw)
    b = P.id_col(A, k, t_reg=1e-4, **kw)
    assert torch.equal(a.J, b.J)
    ea = P.id_error(A, a.J, a.T, a.kout, k).cpu().numpy()
    eb = P.id_error(A, b.J, b.T, b.kout, k).cpu().numpy()
    ra, rb = np.sqrt(ea[0] / ea[1]), np.sqrt(eb[0] / eb[1])
    say(f"  rel fro error plain {ra:.4e} stabilized {rb:.4e}; max|T| {a.T.abs().max().item():.3g} -> "
        f"{b.T.abs().max().item():.3g}")
    assert np.isfinite(rb) and rb <= 1.02 * ra
    assert b.T.abs().max().item() <= a.T.abs().max().item() * (1 + 1e-3)


def test_full_size_fp32_against_oracle():
    """The same workload against the FP64 oracle (Section 4.1, the Tikhonov form
    with t_reg = 1e-4, after Algorithm 4 with one power step of Section 5.3), the
    sketch matrix drawn on the device and given to both sides:
    * against the oracle's stabilized ID of the device's own sketch: J identical
      on the clear-gap prefix (1e-4);
    * T against the oracle's Tikhonov solve for the device's pivots on the same
      sketch, within max(1e-3, 50 cond u32) relative Frobenius, cond that of the
      regularized least-squares system [S11; lam I] (at most about sqrt(k) / t_reg);
    * the ID error within 1.05x of the oracle's stabilized ID on its own FP64
      sketch of the same input and sketch matrix."""
    m, n, k, p, q, treg = 20000, 10000, 200, 10, 1, 1e-4
    say(f"stabilized T full size fp32 {m}x{n} k={k} against the oracle")
    sig = (np.arange(min(m, n), dtype=np.float64) + 1.0) ** -2.0
    A = synth.lowrank_torch(m, n, sig, seed=441, device="cuda").to(torch.float32).contiguous()
    om = P.gaussian(k + p, m, seed=77, dtype=torch.float32)
    got = P.id_col(A, k, p=p, q=q, omega=om, t_reg=treg)
    J = got.J.cpu().numpy()
    check_perm(J, n)
    Yt = P.sketch(A, k, p=p, q=q, omega=om).cpu().numpy().astype(np.float64)
    ref_y = oracle.id_col(Yt.T, k, t_reg=treg)   # the oracle's stabilized ID of the device sketch
    c = clear_prefix(ref_y.qr.gaps, 1e-4)
    say(f"  clear pivots {c} of {k}")
    assert c >= 10
    assert np.array_equal(J[:c], ref_y.J[:c])
    # T for the device's own pivots: the oracle's Tikhonov solve (interp_tikhonov)
    # on S11, S12 from a Householder QR of the sketch's columns J[:k]
    Y = Yt.T
    Q1, S11 = np.linalg.qr(Y[:, J[:k]])
    S12 = Q1.T @ Y[:, J[k:]]
    T_ref = interp_tikhonov(S11, S12, treg)
    lam = tikhonov_weight(S11, treg)
    sv = np.linalg.svd(np.vstack([S11, lam * np.eye(k)]), compute_uv=False)
    cond = sv[0] / sv[-1]
    T = got.T.cpu().numpy().astype(np.float64)
    assert T.shape == T_ref.shape
    dT = np.linalg.norm(T - T_ref) / np.linalg.norm(T_ref)
    bound = max(1e-3, 50.0 * cond * 2.0**-24)
    say(f"  |dT|_F/|T|_F = {dT:.3e} (cond of the regularized system {cond:.3e}, bound {bound:.3e})")
    assert dT <= bound
    A64, om64 = A.cpu().numpy().astype(np.float64), om.cpu().numpy().astype(np.float64)
    ref = oracle.id_col(A64, k, omega=om64, q=q, t_reg=treg)
    del A64
    Jr = torch.as_tensor(ref.J.astype(np.int32), device=A.device)
    Tr = torch.as_tensor(np.ascontiguousarray(ref.T, dtype=np.float32), device=A.device)
    kout = torch.tensor([k, 0], dtype=torch.int32, device=A.device)
    eg = P.id_error(A, got.J, got.T, got.kout, k).cpu().numpy()
    eo = P.id_error(A, Jr, Tr, kout, k).cpu().numpy()
    e_g, e_o = np.sqrt(eg[0] / eg[1]), np.sqrt(eo[0] / eo[1])
    say(f"  e_ID device {e_g:.4e}, FP64 oracle {e_o:.4e}")
    assert e_g <= 1.05 * e_o
