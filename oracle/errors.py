"""Reported error measures. The paper plots relative spectral errors
(Section 6); the headline comparison here is the relative Frobenius error, and
spectral versions are used at small sizes."""
from __future__ import annotations

import numpy as np

from .decomp import vstar_from, w_from


def _norm(X: np.ndarray, kind: str) -> float:
    if kind == "fro":
        return float(np.sqrt((np.asarray(X, dtype=np.float64) ** 2).sum()))
    return float(np.linalg.norm(np.asarray(X, dtype=np.float64), 2))


def rel_fro(E: np.ndarray, A: np.ndarray) -> float:
    return _norm(E, "fro") / _norm(A, "fro")


def e_id(A: np.ndarray, J: np.ndarray, T: np.ndarray, kind: str = "fro") -> float:
    """|A - C V*| / |A| with C = A(:, J(1:k)); only the columns J(k+1:n) carry
    error (the others are reproduced exactly): A(:, J2) - C T."""
    A = np.asarray(A, dtype=np.float64)
    k = T.shape[0]
    E = A[:, J[k:]] - A[:, J[:k]] @ T
    return _norm(E, kind) / _norm(A, kind)


def e_two_sided(A: np.ndarray, J, T, I, Tr, kind: str = "fro") -> float:
    """|A - W A(I(1:k), J(1:k)) V*| / |A| (eq. (two_sided_approx_id))."""
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    k = T.shape[0]
    W = w_from(I, Tr, m)
    Vs = vstar_from(J, T, n)
    E = A - W @ A[np.ix_(I[:k], J[:k])] @ Vs
    return _norm(E, kind) / _norm(A, kind)


def e_cur(A: np.ndarray, C: np.ndarray, U: np.ndarray, R: np.ndarray, kind: str = "fro") -> float:
    A = np.asarray(A, dtype=np.float64)
    return _norm(A - C @ U @ R, kind) / _norm(A, kind)
