"""Truncated column-pivoted Householder QR, written out step by step.

Follows Section 2.2 of the paper (eq. (APQR), (QR) and the partial factorisation
(trunc)): after j steps, A(:,J) = Q1 S1 + Q2 S2 where S1 holds the first j rows
of the upper-trapezoidal factor S. The paper leaves several details open; the
readings taken here (shared with the GPU path, which re-implements them without
sharing code) are:

* pivot: the column of largest remaining 2-norm; ties go to the smallest
  ORIGINAL column index;
* the first k entries of J are the pivots in the order chosen; the remaining
  entries J(k+1:n) list the other columns in increasing index order (the paper
  fixes only that P moves the skeleton to the front; V* = [I T] P* does not
  depend on how the residual columns are ordered as long as T follows J). The
  elimination itself moves columns by swaps, as a column-pivoted QR does;
* Householder sign: alpha = -sgn(x0) |x| with sgn(0) = +1; J, T and all errors
  are invariant to this choice (row signs of S cancel in S11^{-1} S12);
* the remaining column norms are recomputed exactly at every step (no
  downdating): this is the plain definition of the greedy choice;
* rank deficiency (the singular-S11 case of Section 2.3): stop before step j when
  the largest remaining column norm is <= rank_tol * (largest initial column
  norm), and report k_out = j;
* tolerance mode (Section 3, "continue the QR until |E| is below a threshold"):
  stop before step j at the first j with |Y_res|_F <= tol * |Y|_F, where Y_res is
  the not-yet-factored block (its Frobenius norm is the root-sum-square of the
  remaining column norms).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

U64 = 2.0 ** -53


def default_rank_tol(l: int, unit_roundoff: float = U64) -> float:
    """Relative threshold on the pivot norm that declares exact rank deficiency:
    10 * sqrt(l) * u for an l-row matrix in arithmetic with unit roundoff u."""
    return 10.0 * np.sqrt(max(l, 1)) * unit_roundoff


@dataclass
class CPQRResult:
    J: np.ndarray            # int64, pivots in order, then the rest ascending
    S: np.ndarray            # k_out x n, columns of S in the order of J
    k_out: int               # number of Householder steps taken
    pivot_norms: np.ndarray  # |x| of each pivot column at its step (= |S(j,j)|)
    gaps: np.ndarray         # (nu_1 - nu_2)/nu_1 at each step (best vs runner-up)
    stop: str = "k"          # "k" | "rank" | "tol"
    res_fro: list = field(default_factory=list)  # |Y_res|_F before each step


def cpqr(Y: np.ndarray, kmax: int, tol: float | None = None,
         rank_tol: float | None = None, pivot: bool = True) -> CPQRResult:
    """Run up to ``kmax`` steps of column-pivoted Householder QR on ``Y``.

    ``tol`` switches on tolerance mode (relative Frobenius residual).
    ``pivot=False`` keeps the natural column order (unpivoted Householder QR,
    used for the least-squares solve of the CUR factor U)."""
    Y = np.array(Y, dtype=np.float64, copy=True)
    l, n = Y.shape
    kmax = int(min(kmax, l, n))
    if rank_tol is None:
        rank_tol = default_rank_tol(l)
    perm = np.arange(n, dtype=np.int64)
    y_fro = float(np.sqrt((Y ** 2).sum()))
    nu0 = float(np.sqrt((Y ** 2).sum(axis=0)).max()) if n > 0 else 0.0
    pivot_norms, gaps, res_fro = [], [], []
    stop = "k"
    j = 0
    while j < kmax:
        # (a) exact norms of the trailing parts of the remaining columns
        nu = np.sqrt((Y[j:, j:] ** 2).sum(axis=0))
        res = float(np.sqrt((nu ** 2).sum()))
        res_fro.append(res)
        if tol is not None and res <= tol * y_fro:
            stop = "tol"
            break
        if pivot:
            if nu.max() <= rank_tol * nu0:
                stop = "rank"
                break
            # (b) argmax, ties -> smallest original index
            best = nu.max()
            cands = np.flatnonzero(nu == best)
            pos = j + cands[np.argmin(perm[j + cands])]
            srt = np.sort(nu)[::-1]
            gaps.append(float((srt[0] - srt[1]) / srt[0]) if len(srt) > 1 and srt[0] > 0 else 1.0)
            # (c) swap columns j <-> pos
            if pos != j:
                Y[:, [j, pos]] = Y[:, [pos, j]]
                perm[[j, pos]] = perm[[pos, j]]
        else:
            if nu[0] <= rank_tol * nu0:
                stop = "rank"
                break
            gaps.append(float("nan"))
        # (d) Householder reflector that maps x = Y[j:, j] to alpha e_1
        x = Y[j:, j].copy()
        normx = float(np.sqrt((x ** 2).sum()))
        alpha = -normx if x[0] >= 0 else normx
        v = x.copy()
        v[0] -= alpha
        vv = float(v @ v)
        if vv > 0.0:
            w = (v @ Y[j:, j:]) * (2.0 / vv)
            Y[j:, j:] -= np.outer(v, w)
        Y[j, j] = alpha
        Y[j + 1:, j] = 0.0
        pivot_norms.append(normx)
        j += 1
    # present S by original column, then in the order [pivots, rest ascending]
    S_orig = np.zeros((j, n))
    S_orig[:, perm] = Y[:j, :]
    J = np.concatenate([perm[:j], np.sort(perm[j:])])
    return CPQRResult(J=J, S=S_orig[:, J], k_out=j,
                      pivot_norms=np.array(pivot_norms), gaps=np.array(gaps),
                      stop=stop, res_fro=res_fro)
