"""Pins for the oracle's stabilized interpolation matrix (Section 4.1, eq.
(lsqr_for_T) with a Tikhonov term): each check fixes the result by a route
other than the oracle's own SVD filter factors."""
import numpy as np
import pytest

import synth
from oracle import cpqr, id_col, back_substitute
from oracle.stabilized import interp_tikhonov, tikhonov_weight


def _graded_triangle(k, decay, seed):
    """An upper-triangular S11 with singular values spread over `decay` decades
    and an S12 next to it, as a column-pivoted QR produces them."""
    A = synth.lowrank(3 * k, 3 * k, synth.sigma_exp(3 * k, decay), seed=seed)
    res = cpqr(A, k)
    return res.S[:, :k], res.S[:, k:]


def test_stacked_least_squares():
    """The minimizer of |S11 U - S12|^2 + lam^2 |U|^2 is the least-squares
    solution of [S11; lam I] U = [S12; 0], here by LAPACK's lstsq."""
    S11, S12 = _graded_triangle(12, 8.0, seed=301)
    for delta in (1e-1, 1e-3, 1e-6):
        lam = tikhonov_weight(S11, delta)
        k, r = S12.shape
        M = np.vstack([S11, lam * np.eye(k)])
        B = np.vstack([S12, np.zeros((k, r))])
        T_ls = np.linalg.lstsq(M, B, rcond=None)[0]
        T = interp_tikhonov(S11, S12, delta)
        assert np.abs(T - T_ls).max() <= 1e-9 * max(1.0, np.abs(T_ls).max())


def test_stationarity():
    """The gradient of the regularized objective vanishes at T:
    S11^T (S11 T - S12) + lam^2 T = 0."""
    S11, S12 = _graded_triangle(15, 6.0, seed=302)
    delta = 1e-2
    lam = tikhonov_weight(S11, delta)
    T = interp_tikhonov(S11, S12, delta)
    g = S11.T @ (S11 @ T - S12) + lam * lam * T
    scale = np.linalg.norm(S11, 2) * np.linalg.norm(S12, 2)
    assert np.abs(g).max() <= 1e-12 * scale


def test_diagonal_closed_form():
    """Diagonal S11 = diag(d): T(i, j) = d_i S12(i, j) / (d_i^2 + lam^2), with lam
    = delta max |d_i|."""
    d = np.array([3.0, -2.0, 0.5, 1e-4, 7e-9])
    S12 = np.arange(15, dtype=np.float64).reshape(5, 3) - 4.0
    delta = 1e-3
    lam = delta * 3.0
    T = interp_tikhonov(np.diag(d), S12, delta)
    expect = (d / (d * d + lam * lam))[:, None] * S12
    assert np.allclose(T, expect, rtol=1e-13, atol=0.0)
    assert tikhonov_weight(np.diag(d), delta) == pytest.approx(lam, rel=1e-15)


def test_weight_is_the_first_pivot():
    """For a column-pivoted QR the largest column norm of S11 is |S11(1, 1)|."""
    S11, _ = _graded_triangle(10, 5.0, seed=303)
    assert tikhonov_weight(S11, 1.0) == pytest.approx(abs(S11[0, 0]), rel=1e-12)


def test_zero_weight_limit_is_the_triangular_solve():
    """delta -> 0 gives back S11^{-1} S12 (the plain back-substitution); once lam
    is well below the smallest singular value of S11 (here about 1e-4 of the
    largest) the difference shrinks like delta^2."""
    S11, S12 = _graded_triangle(10, 1.0, seed=304)
    T0 = back_substitute(S11, S12)
    d1 = np.abs(interp_tikhonov(S11, S12, 1e-6) - T0).max()
    d2 = np.abs(interp_tikhonov(S11, S12, 1e-7) - T0).max()
    assert d2 <= 2e-2 * d1 + 1e-13
    assert np.abs(interp_tikhonov(S11, S12, 1e-9) - T0).max() <= 1e-9 * max(1.0, np.abs(T0).max())


def test_norm_bound():
    """s / (s^2 + lam^2) <= 1 / (2 lam), so |T|_2 <= |S12|_2 / (2 lam) however
    ill-conditioned S11 is; the unregularized solve on a nearly singular
    triangle exceeds that bound by orders of magnitude."""
    k = 8
    S11 = np.triu(np.ones((k, k)))
    S11[np.arange(k), np.arange(k)] = np.logspace(0, -12, k)
    S12 = np.ones((k, 5))
    delta = 1e-4
    lam = tikhonov_weight(S11, delta)
    T = interp_tikhonov(S11, S12, delta)
    bound = np.linalg.norm(S12, 2) / (2.0 * lam)
    assert np.linalg.norm(T, 2) <= bound * (1 + 1e-12)
    assert np.linalg.norm(back_substitute(S11, S12), 2) > 1e3 * bound


def test_id_col_with_t_reg():
    """The ID path takes the stabilized T on the same pivots; its approximation
    error stays at the rank-k level for a small delta."""
    A = synth.lowrank(60, 50, synth.sigma_exp(50, 6.0), seed=305)
    k = 12
    plain = id_col(A, k)
    reg = id_col(A, k, t_reg=1e-6)
    assert np.array_equal(plain.J, reg.J)
    S = plain.qr.S
    assert np.abs(reg.T - interp_tikhonov(S[:, :k], S[:, k:], 1e-6)).max() == 0.0
    C = A[:, plain.J[:k]]
    e0 = np.linalg.norm(A[:, plain.J[k:]] - C @ plain.T)
    e1 = np.linalg.norm(A[:, reg.J[k:]] - C @ reg.T)
    assert e1 <= 1.5 * e0 + 1e-12 * np.linalg.norm(A)


# ---------------------------------------------------------------------------
# Truncated-SVD pseudo-inverse of S11 (Section 4.1)
# ---------------------------------------------------------------------------
def _thr_between(s, i):
    """A relative threshold strictly between s[i] / s[0] and s[i-1] / s[0]."""
    return float(np.sqrt(s[i] * s[i - 1])) / float(s[0])


def test_tsvd_matches_lapack_lstsq_rcond():
    """With the cut between two singular values, T is LAPACK's minimum-norm
    least-squares solution (gelsd through numpy's lstsq) with rcond = thr, which
    drops the singular values below rcond times the largest."""
    from oracle.stabilized import interp_tsvd
    S11, S12 = _graded_triangle(14, 10.0, seed=311)
    s = np.linalg.svd(S11, compute_uv=False)
    for i in (4, 9, 13):
        thr = _thr_between(s, i)
        T = interp_tsvd(S11, S12, thr)
        T_ls = np.linalg.lstsq(S11, S12, rcond=thr)[0]
        assert np.abs(T - T_ls).max() <= 1e-9 * max(1.0, np.abs(T_ls).max())


def test_tsvd_without_truncation_is_the_inverse():
    """Nothing dropped: T = S11^{-1} S12, here by LU (numpy.linalg.solve) and by
    the oracle's own back-substitution."""
    from oracle.stabilized import interp_tsvd
    S11, S12 = _graded_triangle(10, 2.0, seed=312)
    T = interp_tsvd(S11, S12, 1e-14)
    T_lu = np.linalg.solve(S11, S12)
    assert np.abs(T - T_lu).max() <= 1e-10 * max(1.0, np.abs(T_lu).max())
    assert np.abs(T - back_substitute(S11, S12)).max() <= 1e-10 * max(1.0, np.abs(T_lu).max())


def test_tsvd_diagonal_closed_form():
    """S11 = diag(d): row i of T is S12(i, :) / d_i where d_i >= thr max|d|,
    zero elsewhere."""
    from oracle.stabilized import interp_tsvd
    d = np.array([5.0, 3.0, 1e-3, 2.0, 1e-6, 0.5])
    rng = np.random.default_rng(313)
    S12 = rng.standard_normal((6, 4))
    T = interp_tsvd(np.diag(d), S12, 1e-2)
    want = np.where((d >= 0.05)[:, None], S12 / d[:, None], 0.0)
    assert np.abs(T - want).max() <= 1e-14 * np.abs(want).max()


def test_tsvd_exact_null_space():
    """S11 of rank 3 (two zero singular values, built from random orthogonal
    factors): T has no component in the null space of S11, and S11 T is the
    projection of S12 onto the range of S11."""
    from oracle.stabilized import interp_tsvd
    rng = np.random.default_rng(314)
    Q = np.linalg.qr(rng.standard_normal((5, 5)))[0]
    Z = np.linalg.qr(rng.standard_normal((5, 5)))[0]
    S11 = Q @ np.diag([3.0, 2.0, 1.0, 0.0, 0.0]) @ Z.T
    S12 = rng.standard_normal((5, 7))
    T = interp_tsvd(S11, S12, 1e-8)
    assert np.abs(Z[:, 3:].T @ T).max() <= 1e-12
    P = Q[:, :3] @ Q[:, :3].T
    assert np.abs(S11 @ T - P @ S12).max() <= 1e-12


def test_id_col_tsvd_threshold_small_equals_plain():
    """The column ID with a negligible threshold gives the plain T (Section 2.3,
    eq. (S11T=S12)); a threshold inside the spectrum of S11 changes it."""
    A = synth.lowrank(300, 200, synth.sigma_exp(200, 5.0), seed=315)
    plain = id_col(A, 20)
    stab = id_col(A, 20, t_svd=1e-15)
    assert np.array_equal(plain.J, stab.J)
    assert np.abs(stab.T - plain.T).max() <= 1e-9 * max(1.0, np.abs(plain.T).max())
    cut = id_col(A, 20, t_svd=1e-2)
    assert np.abs(cut.T - plain.T).max() > 1e-6
