"""Column ID, row ID, two-sided ID and CUR-ID, deterministic or sketched.

* Column ID (Section 2.3, eq. (S11T=S12) and (column_approx_id2); Algorithm 1):
  k steps of CPQR give J and S1 = [S11 S12]; T solves S11 T = S12 and
  V* = [I_k T] P*, so A ~ A(:, J(1:k)) V*.
* Row ID (remark closing Section 2.3): the column ID of A^T.
* Two-sided ID (Section 2.4, eq. (boat); Algorithm 2): a full-rank ID of C^T,
  C = A(:, J(1:k)), gives I and W with C = W C(I(1:k), :).
* CUR-ID (Section 3, eq. (choice_C_and_R) and (defU); Algorithm 3):
  C = A(:, J(1:k)), R = A(I(1:k), :), U = V* R^+ as the least-squares solution of
  U R = V* (Section 4.3), computed from a Householder QR of R^T.
* Sketch (Section 5.1, eq. (Y=OmegaA); Algorithm 4): Y = Omega A, then the same
  k-step CPQR on Y. Algorithm 4 writes a full pivoted QR of Y followed by
  dropping p rows of S; the first k steps of a pivoted QR do not depend on the
  later ones, so k steps are taken.
* Power scheme (Section 5.3, the orthonormalised steps (2a)-(2e)):
  Y = Omega A; q times: Y <- orth(Y) A^T; Y <- orth(Y) A, orth taken as a row
  orthonormal basis from the Householder QR of Y^T.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .cpqr import cpqr, CPQRResult
from .backsub import back_substitute
from .stabilized import interp_tikhonov, interp_tsvd


def orth(Y: np.ndarray) -> np.ndarray:
    """Rows forming an orthonormal basis of the row space of Y (no pivoting):
    Q^T from the reduced QR  Y^T = Q R."""
    q, _ = np.linalg.qr(np.asarray(Y, dtype=np.float64).T, mode="reduced")
    return q.T


def sketch(A: np.ndarray, omega: np.ndarray, q: int = 0) -> np.ndarray:
    """Y = Omega A followed by ``q`` orthonormalised power steps."""
    A = np.asarray(A, dtype=np.float64)
    Y = np.asarray(omega, dtype=np.float64) @ A
    for _ in range(int(q)):
        Y = orth(Y) @ A.T
        Y = orth(Y) @ A
    return Y


@dataclass
class IDResult:
    J: np.ndarray      # full permutation, skeleton first
    T: np.ndarray      # k x (n-k)
    k: int             # rank actually produced (k_out)
    qr: CPQRResult
    Y: np.ndarray      # the matrix the CPQR ran on (A itself, or the sketch)


def _id_from_y(Y: np.ndarray, k: int, tol, rank_tol, t_reg: float = 0.0, t_svd: float = 0.0) -> IDResult:
    res = cpqr(Y, k, tol=tol, rank_tol=rank_tol)
    kk = res.k_out
    S11 = res.S[:, :kk]
    S12 = res.S[:, kk:]
    if kk == 0:
        T = np.zeros((0, Y.shape[1]))
    elif t_reg > 0.0:   # the stabilized T of Section 4.1 (Tikhonov form)
        T = interp_tikhonov(S11[:kk], S12[:kk], t_reg)
    elif t_svd > 0.0:   # the stabilized T of Section 4.1 (truncated SVD of S11)
        T = interp_tsvd(S11[:kk], S12[:kk], t_svd)
    else:
        T = back_substitute(S11, S12)
    return IDResult(J=res.J, T=T, k=kk, qr=res, Y=Y)


def id_col(A: np.ndarray, k: int, omega: np.ndarray | None = None, q: int = 0,
           tol: float | None = None, rank_tol: float | None = None, t_reg: float = 0.0,
           t_svd: float = 0.0) -> IDResult:
    """Rank-k column ID of A (Algorithm 1), or of its sketch when ``omega`` is
    given (Algorithm 4 with the power scheme of Section 5.3). ``t_reg > 0`` takes
    the Tikhonov-stabilized T (oracle.stabilized) with delta = t_reg; ``t_svd >
    0`` the truncated-SVD T with relative threshold t_svd."""
    A = np.asarray(A, dtype=np.float64)
    Y = A if omega is None else sketch(A, omega, q)
    return _id_from_y(Y, k, tol, rank_tol, t_reg, t_svd)


def id_row(A: np.ndarray, k: int, omega: np.ndarray | None = None, q: int = 0,
           tol: float | None = None, rank_tol: float | None = None, t_reg: float = 0.0,
           t_svd: float = 0.0) -> IDResult:
    """Row ID A ~ W A(I(1:k), :): the column ID of A^T. ``J`` of the result is
    the row index vector I, ``T`` the row interpolation matrix."""
    return id_col(np.asarray(A, dtype=np.float64).T, k, omega=omega, q=q, tol=tol,
                  rank_tol=rank_tol, t_reg=t_reg, t_svd=t_svd)


def vstar_from(J: np.ndarray, T: np.ndarray, n: int) -> np.ndarray:
    """V* = [I_k T] P* (k x n): column J[s] is e_s for s < k, column J[k+t] is
    T[:, t]."""
    k = T.shape[0]
    V = np.zeros((k, n))
    V[np.arange(k), J[:k]] = 1.0
    V[:, J[k:]] = T
    return V


def w_from(I: np.ndarray, Tr: np.ndarray, m: int) -> np.ndarray:
    """W = P [I_k; Tr^T] (m x k): row I[r] is e_r^T for r < k, row I[k+t] is
    Tr[:, t]^T (the permutation places row r of [I; Tr^T] at I[r])."""
    k = Tr.shape[0]
    W = np.zeros((m, k))
    W[I[:k], np.arange(k)] = 1.0
    W[I[k:], :] = Tr.T
    return W


@dataclass
class TwoSidedResult:
    col: IDResult      # column ID of A (J, T)
    row: IDResult      # full-rank ID of C^T (I = row.J, T_r = row.T)
    C: np.ndarray


def two_sided(A: np.ndarray, k: int, omega: np.ndarray | None = None, q: int = 0,
              tol: float | None = None, rank_tol: float | None = None,
              row_rank_tol: float | None = None, t_reg: float = 0.0, t_svd: float = 0.0) -> TwoSidedResult:
    """Algorithm 2: column ID of A, then a full-rank ID of C^T (k steps of CPQR on
    the k x m matrix C^T). ``t_reg`` or ``t_svd`` stabilizes both interpolation
    matrices."""
    A = np.asarray(A, dtype=np.float64)
    col = id_col(A, k, omega=omega, q=q, tol=tol, rank_tol=rank_tol, t_reg=t_reg, t_svd=t_svd)
    C = A[:, col.J[:col.k]]
    row = _id_from_y(C.T, col.k, None, row_rank_tol, t_reg, t_svd)
    return TwoSidedResult(col=col, row=row, C=C)


@dataclass
class CURResult:
    ts: TwoSidedResult
    C: np.ndarray
    U: np.ndarray
    R: np.ndarray


def cur_u(R: np.ndarray, Vstar: np.ndarray) -> np.ndarray:
    """U = argmin_X |X R - V*|_F, from the Householder QR of R^T = Q S:
    X^T = S^{-1} Q^T V (V = V*^T), solved by back-substitution."""
    Q, S = np.linalg.qr(np.asarray(R, dtype=np.float64).T, mode="reduced")
    return back_substitute(S, Q.T @ np.asarray(Vstar, dtype=np.float64).T).T


def corrected_rhs(A: np.ndarray, C: np.ndarray, Vstar: np.ndarray) -> np.ndarray:
    """The right-hand side of the error-corrected system for U (Section 4.3,
    eq. (cur_ur_sys2)): V* + C^+ E with E = A - C V* the column-ID error
    (eq. (id_error)); C^+ E is the least-squares solution of C X = E."""
    A = np.asarray(A, dtype=np.float64)
    C = np.asarray(C, dtype=np.float64)
    E = A - C @ Vstar
    return Vstar + np.linalg.lstsq(C, E, rcond=None)[0]


def cur(A: np.ndarray, k: int, omega: np.ndarray | None = None, q: int = 0,
        tol: float | None = None, rank_tol: float | None = None,
        row_rank_tol: float | None = None, u_correct: bool = False, t_reg: float = 0.0,
        t_svd: float = 0.0) -> CURResult:
    """Algorithm 3 (CUR-ID): C = A(:, J(1:k)), R = A(I(1:k), :), U = V* R^+;
    with ``u_correct`` U solves U R = V* + C^+ E instead (Section 4.3)."""
    A = np.asarray(A, dtype=np.float64)
    ts = two_sided(A, k, omega=omega, q=q, tol=tol, rank_tol=rank_tol,
                   row_rank_tol=row_rank_tol, t_reg=t_reg, t_svd=t_svd)
    n = A.shape[1]
    kr = ts.row.k
    R = A[ts.row.J[:kr], :]
    Vs = vstar_from(ts.col.J, ts.col.T, n)
    rhs = corrected_rhs(A, ts.C, Vs) if u_correct else Vs
    U = cur_u(R, rhs)
    return CURResult(ts=ts, C=ts.C, U=U, R=R)
