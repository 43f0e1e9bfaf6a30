"""Subsampled randomized Hadamard sketch: the real counterpart of the
subsampled random Fourier transform of Section 5.2, eq. (def_srft).

THIS MODULE IS TEST INFRASTRUCTURE (see the package header).

The paper's structured sketch matrix is sqrt(m/l) R F D (F the unitary DFT, D a
diagonal of random unit-modulus entries, R the rows s_0 .. s_{l-1} of the
identity, drawn without replacement). The real variant built here replaces F by
the orthonormal Walsh-Hadamard matrix of order m' (the smallest power of two
>= m; A is extended by zero rows to m'), whose entry (s, i) is
(-1)^popcount(s & i) / sqrt(m') (Sylvester's construction), and D by random
signs d_i = +-1. The factors combine to

    Omega(r, i) = l^(-1/2) (-1)^popcount(s_r & i) d_i,    r < l, i < m.

``srht_omega`` writes that definition out entry by entry; ``srht_sketch`` forms
Omega A by a fast Walsh-Hadamard transform of the signed, zero-extended columns
(butterflies (x, y) -> (x + y, x - y) at strides 1, 2, 4, ...) and keeps the
sampled rows. The signs and rows are inputs (drawn by ``synth.srht_draws``).
"""
from __future__ import annotations

import numpy as np


def padded_order(m: int) -> int:
    """m': the smallest power of two >= m."""
    p = 1
    while p < m:
        p *= 2
    return p


def hadamard_sign(s: np.ndarray, i: np.ndarray) -> np.ndarray:
    """(-1)^popcount(s & i), elementwise with broadcasting (entries of the
    unnormalised Sylvester-Hadamard matrix)."""
    v = np.bitwise_and(np.asarray(s, dtype=np.int64), np.asarray(i, dtype=np.int64))
    par = np.zeros(v.shape, dtype=np.int64)
    while np.any(v):
        par ^= v & 1
        v = v >> 1
    return 1.0 - 2.0 * par


def srht_omega(m: int, rows, signs) -> np.ndarray:
    """The l x m sketch matrix, entry by entry from its definition."""
    rows = np.asarray(rows, dtype=np.int64)
    d = np.where(np.asarray(signs)[:m] < 0, -1.0, 1.0)
    l = rows.size
    return hadamard_sign(rows[:, None], np.arange(m)[None, :]) * d[None, :] / np.sqrt(l)


def fwht(X: np.ndarray) -> np.ndarray:
    """Unnormalised Walsh-Hadamard transform along axis 0 (length a power of
    two): H X with H(s, i) = (-1)^popcount(s & i)."""
    Z = np.array(X, dtype=np.float64, copy=True)
    n = Z.shape[0]
    h = 1
    while h < n:
        Z = Z.reshape((n // (2 * h), 2, h) + Z.shape[1:])
        a = Z[:, 0].copy()
        b = Z[:, 1].copy()
        Z[:, 0] = a + b
        Z[:, 1] = a - b
        Z = Z.reshape((n,) + Z.shape[3:])
        h *= 2
    return Z


def srht_sketch(A: np.ndarray, rows, signs) -> np.ndarray:
    """Y = Omega A (l x n) by the fast transform."""
    A = np.asarray(A, dtype=np.float64)
    m = A.shape[0]
    mp = padded_order(m)
    rows = np.asarray(rows, dtype=np.int64)
    d = np.where(np.asarray(signs)[:m] < 0, -1.0, 1.0)
    Z = np.zeros((mp,) + A.shape[1:])
    Z[:m] = d.reshape((m,) + (1,) * (A.ndim - 1)) * A
    return fwht(Z)[rows] / np.sqrt(rows.size)
