"""Pins for the oracle's truncated column-pivoted QR (Section 2.2).

Each test checks the oracle against something other than itself: a brute-force
greedy definition, LAPACK's pivoted QR, closed forms on structured inputs, and
invariances the paper's construction implies."""
import itertools

import numpy as np
import pytest
import scipy.linalg

import synth
from oracle import cpqr, default_rank_tol


def _well_separated(l, n, seed, decay=0.7):
    """Columns with geometrically spread scales -> well-separated greedy gaps."""
    g = synth.rng(seed)
    Y = g.standard_normal((l, n)) * (decay ** np.arange(n))[g.permutation(n)]
    return Y


@pytest.mark.parametrize("shape,seed", [((8, 12), 1), ((12, 8), 2), ((16, 16), 3), ((5, 14), 4)])
def test_pivots_match_brute_force_greedy(shape, seed):
    """Pivot j is the column farthest from the span of the pivots already taken
    (distance by an independent least-squares solve on the ORIGINAL matrix)."""
    Y = _well_separated(*shape, seed)
    k = min(shape) - 1
    res = cpqr(Y, k)
    assert res.k_out == k
    for j in range(k):
        chosen = res.J[:j]
        best, best_c = -1.0, None
        for c in range(shape[1]):
            if c in chosen:
                continue
            if j == 0:
                d = np.linalg.norm(Y[:, c])
            else:
                coef = np.linalg.lstsq(Y[:, chosen], Y[:, c], rcond=None)[0]
                d = np.linalg.norm(Y[:, c] - Y[:, chosen] @ coef)
            if d > best:
                best, best_c = d, c
        assert res.J[j] == best_c, f"step {j}"
        # |S(j,j)| equals that distance
        assert abs(res.pivot_norms[j] - best) <= 1e-10 * max(best, 1e-300)
        assert abs(abs(res.S[j, j]) - best) <= 1e-10 * max(best, 1e-300)


def test_first_pivot_is_largest_column():
    Y = synth.rng(5).standard_normal((6, 30))
    res = cpqr(Y, 1)
    assert res.J[0] == int(np.argmax(np.linalg.norm(Y, axis=0)))


def test_diagonal_input_sorted_pivots_and_exact_tail():
    d = np.array([3.0, -7.0, 0.5, 11.0, 2.0, -0.25, 5.0])
    m, n = 9, 7
    A = np.zeros((m, n))
    A[np.arange(n), np.arange(n)] = d
    k = 4
    res = cpqr(A, k)
    order = np.argsort(-np.abs(d), kind="stable")
    assert list(res.J[:k]) == list(order[:k])
    # S11 diagonal (up to sign) = the selected |d|, S12 = 0 -> T = 0
    assert np.allclose(np.abs(np.diag(res.S[:, :k])), np.abs(d[order[:k]]), rtol=0, atol=1e-14)
    assert np.abs(res.S[:, k:]).max() == 0.0


def test_mutually_orthogonal_columns_give_zero_coupling():
    Q = synth.haar_orthonormal(20, 10, 6)
    A = Q * np.linspace(1.0, 3.0, 10)
    res = cpqr(A, 4)
    assert np.abs(res.S[:, 4:]).max() < 1e-13


@pytest.mark.parametrize("seed", [11, 12, 13])
def test_agrees_with_lapack_pivoted_qr_where_gaps_are_clear(seed):
    Y = _well_separated(30, 25, seed, decay=0.8)
    k = 15
    res = cpqr(Y, k)
    _, _, P = scipy.linalg.qr(Y, pivoting=True, mode="economic")
    clear = 0
    for j in range(k):
        if res.gaps[j] < 1e-8:
            break
        clear += 1
    assert clear >= 5
    assert list(res.J[:clear]) == list(P[:clear])


def test_ties_go_to_smallest_original_index():
    Y = np.zeros((4, 5))
    Y[0, 0] = 1.0
    Y[1, 3] = 2.0
    Y[2, 1] = 2.0   # ties with column 3 -> column 1 wins
    Y[3, 4] = 0.5
    res = cpqr(Y, 3)
    assert list(res.J[:3]) == [1, 3, 0]


def test_rank_deficiency_stops_at_rank():
    r = 5
    A = synth.lowrank(40, 30, synth.sigma_exp(r, 2.0), seed=21, rank=r)
    res = cpqr(A, r + 3)
    assert res.k_out == r and res.stop == "rank"
    assert default_rank_tol(40) < 1e-12


def test_tolerance_mode_stops_at_first_rank_meeting_tol():
    A = synth.lowrank(60, 50, synth.sigma_exp(50, 4.0), seed=22)
    tol = 1e-3
    res = cpqr(A, 50, tol=tol)
    assert res.stop == "tol"
    k = res.k_out
    full = cpqr(A, 50)
    fro = np.linalg.norm(A)
    # residual Frobenius norms before each step, recomputed from the explicit
    # rank-j factorisation Q1 S1 of an independent library QR with the same pivots
    for j, want in [(k, True), (k - 1, False)]:
        Jj = full.J[:j]
        if j == 0:
            resid = fro
        else:
            coef = np.linalg.lstsq(A[:, Jj], A, rcond=None)[0]
            resid = np.linalg.norm(A - A[:, Jj] @ coef)
        assert (resid <= tol * fro) == want


def test_truncated_qr_error_identity():
    """A - C V* = Q2 S22 (eq. (id_error)): |A(:,J2) - C T|_F equals the Frobenius
    norm of the unfactored block after k steps."""
    from oracle import id_col, e_id
    A = synth.lowrank(80, 60, synth.sigma_exp(60, 6.0), seed=23)
    k = 12
    ident = id_col(A, k)
    nxt = cpqr(A, k + 1)
    lhs = e_id(A, ident.J, ident.T) * np.linalg.norm(A)
    assert abs(lhs - nxt.res_fro[k]) <= 1e-12 * nxt.res_fro[k] + 1e-15


def test_left_orthogonal_invariance():
    """CPQR sees only column norms and distances, which Q Y preserves."""
    Y = _well_separated(20, 30, 24, decay=0.85)
    Q = synth.haar_orthonormal(20, 20, 25)
    a, b = cpqr(Y, 10), cpqr(Q @ Y, 10)
    assert list(a.J) == list(b.J)
    from oracle import back_substitute
    Ta = back_substitute(a.S[:, :10], a.S[:, 10:])
    Tb = back_substitute(b.S[:, :10], b.S[:, 10:])
    assert np.abs(Ta - Tb).max() <= 1e-9 * max(1.0, np.abs(Ta).max())


def test_power_of_two_scaling_is_bitwise_invariant():
    Y = _well_separated(15, 25, 26)
    a, b = cpqr(Y, 8), cpqr(Y * 2.0 ** 7, 8)
    assert np.array_equal(a.J, b.J)
    assert np.array_equal(a.S * 2.0 ** 7, b.S)


def test_permutation_layout():
    Y = _well_separated(10, 30, 28)
    res = cpqr(Y, 6)
    assert sorted(res.J) == list(range(30))
    assert list(res.J[6:]) == sorted(res.J[6:])
    # S columns follow J: S11 upper triangular, and Y(:,J) = Q1 S1 + residual
    assert np.abs(np.tril(res.S[:, :6], -1)).max() == 0.0
    Q = np.linalg.lstsq(res.S[:, :6].T, Y[:, res.J[:6]].T, rcond=None)[0].T
    assert np.abs(Q.T @ Q - np.eye(6)).max() < 1e-12
    assert np.abs(Q.T @ Y[:, res.J] - res.S).max() < 1e-12 * np.abs(Y).max()


def test_unpivoted_mode_is_householder_qr():
    Y = synth.rng(27).standard_normal((12, 5))
    res = cpqr(Y, 5, pivot=False)
    assert list(res.J) == list(range(5))
    R = np.linalg.qr(Y, mode="r")
    assert np.allclose(np.abs(res.S[:, :5]), np.abs(R), atol=1e-12)
