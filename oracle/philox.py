"""Philox4x32-10 and the Gaussian sketch matrix drawn from it.

Philox4x32-10 is the counter-based generator of Salmon, Moraes, Dror and Shaw,
"Parallel random numbers: as easy as 1, 2, 3" (SC'11): ten rounds of a bijection
on a 4 x 32-bit counter under a 2 x 32-bit key. One round maps
(c0, c1, c2, c3) to (hi(M1 c2) ^ c1 ^ k0, lo(M1 c2), hi(M0 c0) ^ c3 ^ k1, lo(M0 c0))
with M0 = 0xD2511F53, M1 = 0xCD9E8D57, and the key is advanced by the Weyl
increments (0x9E3779B9, 0xBB67AE85) between rounds.

The sketch matrix Omega (l x m, i.i.d. N(0,1), Section 5.1) is defined element by
element: entry (r, i) has flat index f = r*m + i; the generator is called on
counter (g mod 2^32, g div 2^32, stream, 0) with g = f div 4 and key
(seed mod 2^32, seed div 2^32); its four words (x0, x1, x2, x3) give two
Box-Muller pairs with u1 = (x_a + 1) / 2^32 in (0, 1] and u2 = x_b / 2^32 in [0, 1):
rho = sqrt(-2 ln u1), z = (rho cos 2 pi u2, rho sin 2 pi u2); f mod 4 picks
(pair 0 cos, pair 0 sin, pair 1 cos, pair 1 sin).
"""
from __future__ import annotations

import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = np.uint64(0x9E3779B9)
W1 = np.uint64(0xBB67AE85)
MASK = np.uint64(0xFFFFFFFF)


def philox4x32_10(ctr: np.ndarray, key: np.ndarray) -> np.ndarray:
    """Apply Philox4x32-10 to counters ``ctr`` (N x 4 uint32) under keys ``key``
    (N x 2 or 2 uint32). Returns N x 4 uint32."""
    c = np.asarray(ctr, dtype=np.uint64).reshape(-1, 4).copy()
    k = np.broadcast_to(np.asarray(key, dtype=np.uint64).reshape(-1, 2), (c.shape[0], 2)).copy()
    for rnd in range(10):
        if rnd > 0:
            k[:, 0] = (k[:, 0] + W0) & MASK
            k[:, 1] = (k[:, 1] + W1) & MASK
        p0 = c[:, 0] * M0          # < 2^64, exact in uint64
        p1 = c[:, 2] * M1
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK
        c = np.stack([hi1 ^ c[:, 1] ^ k[:, 0], lo1, hi0 ^ c[:, 3] ^ k[:, 1], lo0], axis=1)
    return c.astype(np.uint32)


def gaussian_omega(rows: int, cols: int, seed: int, stream: int = 0) -> np.ndarray:
    """Omega (rows x cols, float64) from the element-wise definition above."""
    total = rows * cols
    ngroups = (total + 3) // 4
    g = np.arange(ngroups, dtype=np.uint64)
    ctr = np.stack([g & MASK, g >> np.uint64(32),
                    np.full_like(g, np.uint64(stream) & MASK), np.zeros_like(g)], axis=1)
    key = np.array([np.uint64(seed) & MASK, (np.uint64(seed) >> np.uint64(32)) & MASK],
                   dtype=np.uint64)
    x = philox4x32_10(ctr, key).astype(np.float64)
    scale = 2.0 ** -32
    out = np.empty((ngroups, 4))
    for pair in range(2):
        u1 = (x[:, 2 * pair] + 1.0) * scale
        u2 = x[:, 2 * pair + 1] * scale
        rho = np.sqrt(-2.0 * np.log(u1))
        out[:, 2 * pair] = rho * np.cos(2.0 * np.pi * u2)
        out[:, 2 * pair + 1] = rho * np.sin(2.0 * np.pi * u2)
    return out.reshape(-1)[:total].reshape(rows, cols)
