"""Adaptive-rank column ID of many independent blocks (the tolerance variant of
Section 3, with the randomized sketch of Section 5.1 and Algorithm 4), one block
at a time.

THIS MODULE IS TEST INFRASTRUCTURE (see the package header).

Readings (the paper states the tolerance variant only as "continue until the
residual is below a threshold"):

* One sketch matrix serves every block: Omega (l_cap x m_max, i.i.d. N(0,1)),
  block b uses its leading l x m_b part. Each block still sees a Gaussian
  matrix independent of its data.
* Tolerance mode: the rank is the smallest k with |Y_res|_F <= tol |Y|_F for the
  sketch Y = Omega(:l, :m_b) A_b (the oracle's ``cpqr`` tolerance rule, the
  residual tested before every step and after the last allowed one). The
  sketch estimate is only trusted for k <= l - p, so at most l - p steps are
  taken; when the tolerance is not met by then, l doubles (up to
  l_cap = kmax + p) and the block is sketched and factored again. Starting
  width l_0 = min(32, l_cap); p >= 1. When even l_cap does not meet the
  tolerance the block keeps the l_cap - p steps taken and is flagged.
* Fixed-rank mode (tol is None): l = k + p, k steps.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .decomp import _id_from_y, IDResult

L0 = 32


@dataclass
class AdaptiveResult:
    id: IDResult
    l: int          # sketch width of the final pass
    met: bool       # tolerance reached (always True in fixed-rank mode)


def id_col_adaptive(A: np.ndarray, omega: np.ndarray, p: int, *, tol: float | None = None,
                    kmax: int | None = None, k: int | None = None,
                    rank_tol: float | None = None) -> AdaptiveResult:
    """Column ID of one block with the width-doubling rule above. ``omega`` is
    the shared sketch matrix (at least l_cap x m)."""
    A = np.asarray(A, dtype=np.float64)
    m = A.shape[0]
    om = np.asarray(omega, dtype=np.float64)
    if tol is None:
        l = int(k) + p
        Y = om[:l, :m] @ A
        return AdaptiveResult(_id_from_y(Y, int(k), None, rank_tol), l, True)
    lcap = int(kmax) + p
    l = min(L0, lcap)
    while True:
        Y = om[:l, :m] @ A
        cap = l - p
        # one step beyond the cap, so that the residual after step cap is tested
        r = _id_from_y(Y, cap + 1, tol, rank_tol)
        met = r.qr.stop in ("tol", "rank") and r.k <= cap
        if not met:
            r = _id_from_y(Y, cap, None, rank_tol)
        if met or l >= lcap:
            return AdaptiveResult(r, l, met)
        l = min(2 * l, lcap)


def id_col_batched(blocks, omega: np.ndarray, p: int, **kw) -> list[AdaptiveResult]:
    """``id_col_adaptive`` over a list of blocks."""
    return [id_col_adaptive(B, omega, p, **kw) for B in blocks]
