"""Pins for the oracle's ID / two-sided ID / CUR-ID and the sketch (Sections 2-5)."""
import itertools
import math

import numpy as np
import pytest

import synth
from oracle import (id_col, id_row, two_sided, cur, sketch, orth, vstar_from, w_from,
                    e_id, e_two_sided, e_cur, cpqr)
from oracle.decomp import cur_u


def _spectral(X):
    return float(np.linalg.norm(X, 2))


def test_T_is_the_least_squares_interpolation():
    """T = argmin |Y(:,J1) T - Y(:,J2)| (eq. (lsqr_for_T)), by a library solver."""
    A = synth.lowrank(50, 40, synth.sigma_exp(40, 5.0), seed=31)
    k = 10
    ident = id_col(A, k)
    J1, J2 = ident.J[:k], ident.J[k:]
    T_ls = np.linalg.lstsq(A[:, J1], A[:, J2], rcond=None)[0]
    assert np.abs(ident.T - T_ls).max() <= 1e-9 * max(1.0, np.abs(T_ls).max())


def test_identity_structure_is_exact():
    A = synth.lowrank(30, 25, synth.sigma_exp(25, 3.0), seed=32)
    k = 6
    res = cur(A, k)
    J, I = res.ts.col.J, res.ts.row.J
    assert np.array_equal(res.C, A[:, J[:k]])
    assert np.array_equal(res.R, A[I[:k], :])
    Vs = vstar_from(J, res.ts.col.T, 25)
    assert np.array_equal(Vs[:, J[:k]], np.eye(k))
    W = w_from(I, res.ts.row.T, 30)
    assert np.array_equal(W[I[:k], :], np.eye(k))
    assert sorted(J) == list(range(25)) and sorted(I) == list(range(30))


@pytest.mark.parametrize("m,n,r", [(40, 30, 5), (25, 60, 7)])
def test_exact_rank_r_is_reconstructed(m, n, r):
    A = synth.lowrank(m, n, synth.sigma_pow(r, 1.0), seed=33 + r, rank=r)
    res = cur(A, r)
    ts = res.ts
    assert ts.col.k == r and ts.row.k == r
    assert e_id(A, ts.col.J, ts.col.T) <= 1e-12
    assert e_two_sided(A, ts.col.J, ts.col.T, ts.row.J, ts.row.T) <= 1e-12
    assert e_cur(A, res.C, res.U, res.R) <= 1e-11


def test_row_id_of_C_is_exact():
    """The ID of C^T is a full (not partial) factorisation: C = W C(I(1:k), :)."""
    A = synth.lowrank(70, 50, synth.sigma_exp(50, 8.0), seed=34)
    ts = two_sided(A, 12)
    C = ts.C
    W = w_from(ts.row.J, ts.row.T, 70)
    err = np.linalg.norm(C - W @ C[ts.row.J[:12], :]) / np.linalg.norm(C)
    assert err <= 1e-13


def test_two_sided_adds_no_error():
    """A - C V* = A - W A(I,J) V* (Section 2.4)."""
    A = synth.lowrank(60, 45, synth.sigma_exp(45, 5.0), seed=35)
    ts = two_sided(A, 9)
    e1 = e_id(A, ts.col.J, ts.col.T)
    e2 = e_two_sided(A, ts.col.J, ts.col.T, ts.row.J, ts.row.T)
    assert abs(e1 - e2) <= 1e-10 * e1


@pytest.mark.parametrize("k", [5, 15])
def test_eckart_young_floors(k):
    m, n = 90, 70
    sig = synth.sigma_exp(70, 7.0)
    A = synth.lowrank(m, n, sig, seed=36)
    res = cur(A, k)
    ts = res.ts
    fro_floor = math.sqrt((sig[k:] ** 2).sum() / (sig ** 2).sum())
    assert e_id(A, ts.col.J, ts.col.T) >= fro_floor * (1 - 1e-12)
    assert e_cur(A, res.C, res.U, res.R) >= fro_floor * (1 - 1e-12)
    spec = e_id(A, ts.col.J, ts.col.T, kind="spec")
    assert spec >= sig[k] / sig[0] * (1 - 1e-12)


def test_lemmas_and_corollary():
    """Lemma 3.1 (|A-CUR| <= |E| + |Et|), Lemma 3.2 (Et = P[0; F E]) and the
    corollary (|Et| <= (1+|T|)|E|, |A-CUR| <= (2+|T|)|E|), spectral norm."""
    A = synth.lowrank(80, 60, synth.sigma_logspace(60, -4.0), seed=37)
    k = 10
    res = cur(A, k)
    ts = res.ts
    J, T = ts.col.J, ts.col.T
    I, Tr = ts.row.J, ts.row.T
    Vs = vstar_from(J, T, 60)
    E = A - res.C @ Vs
    W = w_from(I, Tr, 80)
    Et = A - W @ res.R
    # Lemma 3.2: rows I_skel of Et vanish, rows I_res equal E(I_res) - Tr^T E(I_skel)
    assert np.abs(Et[I[:k], :]).max() <= 1e-12 * np.abs(A).max()
    want = E[I[k:], :] - Tr.T @ E[I[:k], :]
    assert np.abs(Et[I[k:], :] - want).max() <= 1e-11 * np.abs(A).max()
    nE, nEt, nT = _spectral(E), _spectral(Et), _spectral(Tr)
    ncur = _spectral(A - res.C @ res.U @ res.R)
    assert ncur <= (nE + nEt) * (1 + 1e-10)
    assert nEt <= (1 + nT) * nE * (1 + 1e-10)
    assert ncur <= (2 + nT) * nE * (1 + 1e-10)


def test_cpqr_skeleton_versus_all_subsets():
    """min over all k-subsets of the ID error lies between the Eckart-Young floor
    and the CPQR skeleton's error (CPQR is greedy, not optimal)."""
    m, n, k = 14, 9, 3
    sig = synth.sigma_exp(9, 2.0)
    A = synth.lowrank(m, n, sig, seed=38)
    floor = math.sqrt((sig[k:] ** 2).sum() / (sig ** 2).sum())
    best = float("inf")
    for J1 in itertools.combinations(range(n), k):
        J1 = list(J1)
        coef = np.linalg.lstsq(A[:, J1], A, rcond=None)[0]
        best = min(best, np.linalg.norm(A - A[:, J1] @ coef) / np.linalg.norm(A))
    ident = id_col(A, k)
    e = e_id(A, ident.J, ident.T)
    assert floor * (1 - 1e-12) <= best <= e * (1 + 1e-12)


def test_U_by_qr_matches_pseudo_inverse():
    A = synth.lowrank(40, 35, synth.sigma_exp(35, 6.0), seed=39)
    res = cur(A, 8)
    Vs = vstar_from(res.ts.col.J, res.ts.col.T, 35)
    U_pinv = Vs @ np.linalg.pinv(res.R)
    assert np.abs(res.U - U_pinv).max() <= 1e-8 * np.abs(U_pinv).max()
    U2 = cur_u(res.R, Vs)
    assert np.array_equal(U2, res.U)


def test_identity_sketch_reduces_to_deterministic():
    A = synth.lowrank(30, 40, synth.sigma_exp(30, 4.0), seed=40)
    a = id_col(A, 8)
    b = id_col(A, 8, omega=np.eye(30), q=0)
    assert np.array_equal(a.J, b.J) and np.array_equal(a.T, b.T)


def test_orthogonal_sketch_gives_same_skeleton():
    A = synth.lowrank(30, 40, synth.sigma_exp(30, 4.0), seed=41)
    a = id_col(A, 8)
    Q = synth.haar_orthonormal(30, 30, 42)
    b = id_col(A, 8, omega=Q, q=0)
    assert np.array_equal(a.J, b.J)
    assert np.abs(a.T - b.T).max() <= 1e-9 * max(1.0, np.abs(a.T).max())


def test_power_of_two_scaling_keeps_skeleton_and_T():
    A = synth.lowrank(50, 40, synth.sigma_exp(40, 4.0), seed=43)
    om = synth.gaussian(18, 50, 44)
    a = id_col(A, 8, omega=om, q=1)
    b = id_col(A * 2.0 ** -20, 8, omega=om, q=1)
    assert np.array_equal(a.J, b.J)
    assert np.abs(a.T - b.T).max() <= 1e-10 * max(1.0, np.abs(a.T).max())


def test_orth_rows_are_orthonormal_and_span_the_rows():
    Y = synth.rng(45).standard_normal((7, 30))
    Q = orth(Y)
    assert np.abs(Q @ Q.T - np.eye(7)).max() <= 1e-14
    # same row space: projecting Y onto rows of Q reproduces Y
    assert np.abs(Y - (Y @ Q.T) @ Q).max() <= 1e-13


def test_power_scheme_row_space():
    """With q=1 the sketch spans the row space of Omega A (A^T A) (eq. (Ypower));
    checked through principal angles on a small, well-conditioned example."""
    A = synth.lowrank(40, 30, synth.sigma_exp(30, 10.0), seed=46)
    om = synth.gaussian(6, 40, 47)
    Y = sketch(A, om, q=1)
    Z = om @ A @ A.T @ A
    qa = np.linalg.qr(Y.T)[0]
    qb = np.linalg.qr(Z.T)[0]
    s = np.linalg.svd(qa.T @ qb, compute_uv=False)
    assert s.min() >= 1 - 1e-10


def test_randomized_id_close_to_deterministic_with_power_step():
    """Probe-level check of the randomized path on a decaying spectrum: error with
    p=10, q=1 is within a small factor of the deterministic error."""
    m, n, k = 300, 200, 20
    A = synth.lowrank(m, n, synth.sigma_pow(200, 2.0), seed=48)
    det = id_col(A, k)
    rnd = id_col(A, k, omega=synth.gaussian(k + 10, m, 49), q=1)
    e_det = e_id(A, det.J, det.T)
    e_rnd = e_id(A, rnd.J, rnd.T)
    assert e_rnd <= 3.0 * e_det


def test_row_id_is_column_id_of_transpose():
    A = synth.lowrank(25, 35, synth.sigma_exp(25, 3.0), seed=50)
    r = id_row(A, 6)
    c = id_col(A.T, 6)
    assert np.array_equal(r.J, c.J) and np.array_equal(r.T, c.T)
    W = w_from(r.J, r.T, 25)
    assert np.array_equal(W[r.J[:6]], np.eye(6))


# ---------------------------------------------------------------------------
# Error-corrected U (Section 4.3, eq. (cur_ur_sys2))
# ---------------------------------------------------------------------------
def test_corrected_u_is_the_frobenius_optimal_u_by_brute_force():
    # tiny case: min_U |A - C U R|_F over all k x k U, solved as one least-squares
    # problem in vec(U) (vec(C U R) = (R^T kron C) vec(U)); the corrected system
    # must reach that optimum, the plain one not below it
    import oracle.decomp as D
    m, n, k = 14, 11, 3
    A = synth.lowrank(m, n, synth.sigma_exp(min(m, n), 1.5), seed=4)
    ref = D.cur(A, k, u_correct=True)
    plain = D.cur(A, k)
    K = np.kron(ref.R.T, ref.C)
    u = np.linalg.lstsq(K, A.reshape(-1, order="F"), rcond=None)[0]
    U_opt = u.reshape(k, k, order="F")
    e_opt = np.linalg.norm(A - ref.C @ U_opt @ ref.R)
    e_cor = np.linalg.norm(A - ref.C @ ref.U @ ref.R)
    e_pl = np.linalg.norm(A - plain.C @ plain.U @ plain.R)
    assert abs(e_cor - e_opt) <= 1e-10 * np.linalg.norm(A)
    assert e_pl >= e_opt * (1 - 1e-12)


def test_corrected_u_equals_c_pinv_a_r_pinv():
    # closed form: V* + C^+ (A - C V*) = C^+ A when C has full column rank, so
    # U = C^+ A R^+
    import oracle.decomp as D
    m, n, k = 60, 45, 7
    A = synth.lowrank(m, n, synth.sigma_exp(min(m, n), 3.0), seed=12)
    ref = D.cur(A, k, u_correct=True)
    U_cf = np.linalg.pinv(ref.C) @ A @ np.linalg.pinv(ref.R)
    assert np.abs(ref.U - U_cf).max() <= 1e-8 * np.abs(U_cf).max()
