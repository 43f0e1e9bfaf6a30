"""Back-substitution for S X = B with S upper triangular (Section 4.1: T is
computed from S11 T = S12 by a backwards solve)."""
from __future__ import annotations

import numpy as np


def back_substitute(S: np.ndarray, B: np.ndarray) -> np.ndarray:
    """Solve S X = B for X, S (k x k) upper triangular, B (k x r).

    Row i of X is (B[i] - S[i, i+1:] X[i+1:]) / S[i, i], taken from the last row
    up; every right-hand side is handled the same way."""
    S = np.asarray(S, dtype=np.float64)
    X = np.array(B, dtype=np.float64, copy=True)
    k = S.shape[0]
    if X.ndim == 1:
        X = X[:, None]
    for i in range(k - 1, -1, -1):
        if i + 1 < k:
            X[i, :] -= S[i, i + 1:] @ X[i + 1:, :]
        X[i, :] /= S[i, i]
    return X
