"""Stabilized interpolation matrix (Section 4.1, eq. (lsqr_for_T)): T as the
least-squares solution of S11 U ~ S12, regularized.

Test infrastructure: only the tests, the smoke check and the bench's CPU
baseline call this module; the library never does.

When S11 is ill-conditioned the paper treats T as the minimizer of
|S11 U - S12| and names two stabilized solutions: a truncated-SVD pseudo-inverse
of S11, or a Tikhonov term added to the minimization. This module gives both.

Truncated SVD: with S11 = Ut diag(s) Vt^T, the terms whose singular value is
below thr times the largest are dropped and

    T = Vt_kept diag(1 / s_kept) Ut_kept^T S12,

the minimum-norm least-squares solution for the truncated S11.

Tikhonov: the minimizer

    T = argmin_U |S11 U - S12|_F^2 + lam^2 |U|_F^2,   lam = delta * max_j |S11(:, j)|_2

is written out from the SVD S11 = Ut diag(s) Vt^T that the paper starts from:
T = Vt diag(s / (s^2 + lam^2)) Ut^T S12 (every singular direction kept, damped
by its filter factor s^2 / (s^2 + lam^2)). The weight lam is relative to the
largest column norm of S11, which for a column-pivoted QR is |S11(1, 1)|, so
the same delta serves any scaling of A. delta = 0 gives back S11^{-1} S12.
"""
from __future__ import annotations

import numpy as np


def tikhonov_weight(S11: np.ndarray, delta: float) -> float:
    """lam = delta times the largest column norm of S11."""
    S11 = np.asarray(S11, dtype=np.float64)
    if S11.size == 0:
        return 0.0
    return float(delta) * float(np.max(np.sqrt(np.sum(S11 * S11, axis=0))))


def interp_tikhonov(S11: np.ndarray, S12: np.ndarray, delta: float) -> np.ndarray:
    """The Tikhonov-regularized T (k x r) for S11 (k x k) and S12 (k x r), in FP64,
    through the SVD of S11 (Section 4.1's stabilized solution of eq.
    (lsqr_for_T) with a regularization term)."""
    S11 = np.asarray(S11, dtype=np.float64)
    S12 = np.asarray(S12, dtype=np.float64)
    k = S11.shape[0]
    if k == 0:
        return np.zeros((0, S12.shape[1]))
    lam = tikhonov_weight(S11, delta)
    Ut, s, Vth = np.linalg.svd(S11)
    filt = s / (s * s + lam * lam)
    return Vth.T @ (filt[:, None] * (Ut.T @ S12))


def interp_tsvd(S11: np.ndarray, S12: np.ndarray, thr: float) -> np.ndarray:
    """The truncated-SVD T (k x r) for S11 (k x k) and S12 (k x r), in FP64
    (Section 4.1's stabilized pseudo-inverse of S11 in eq. (lsqr_for_T)): the
    SVD of S11, the terms with a singular value below thr times the largest
    dropped, T = V D^{-1} U^T S12 over the rest."""
    S11 = np.asarray(S11, dtype=np.float64)
    S12 = np.asarray(S12, dtype=np.float64)
    k = S11.shape[0]
    if k == 0:
        return np.zeros((0, S12.shape[1]))
    Ut, s, Vth = np.linalg.svd(S11)
    keep = s >= float(thr) * s[0] if s[0] > 0 else np.zeros_like(s, dtype=bool)
    keep &= s > 0
    return Vth[keep].T @ ((Ut[:, keep].T @ S12) / s[keep, None])
