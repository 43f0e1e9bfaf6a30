"""Seeded synthetic inputs shared by the tests, the bench and the oracle checks.

This module only draws random numbers and assembles test matrices. It holds none
of the decomposition's arithmetic (no pivoting, no Householder, no triangular
solves), so the oracle and the GPU path can both take their inputs from here
without sharing any part of the method.

Workloads (all synthetic; the paper's own test matrices are synthetic too, and
its image experiment data is not available):

* ``lowrank``: A = U diag(sigma) V^T with U, V the Q factors (diag(R) > 0) of
  seeded N(0,1) matrices -- the construction of the paper's Section 6 test sets
  (random orthonormal factors and a prescribed spectrum).
* ``kernel_blocks``: blocks K_ij = 1/|x_i - y_j| between two seeded point
  clusters in unit cubes whose centres are 4 apart (well-separated interactions).
* ``gaussian``: i.i.d. N(0,1) matrices, used as caller-supplied sketch matrices.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = [
    "rng",
    "haar_orthonormal",
    "lowrank",
    "lowrank_torch",
    "noisy_lowrank_torch",
    "noisy_lowrank_blocks_torch",
    "srht_draws",
    "gaussian",
    "sigma_exp",
    "sigma_pow",
    "sigma_logspace",
    "kernel_block",
    "kernel_block_sizes",
    "kernel_blocks_torch",
    "CONFIGS",
    "Config",
]


def rng(seed: int) -> np.random.Generator:
    """A NumPy generator on the Philox bit generator, keyed by ``seed``."""
    return np.random.Generator(np.random.Philox(int(seed)))


def haar_orthonormal(rows: int, cols: int, seed: int) -> np.ndarray:
    """rows x cols matrix with orthonormal columns, from the QR of N(0,1) data.

    The signs of R's diagonal are moved into Q so the result is unique for the
    draw (and Haar distributed)."""
    g = rng(seed).standard_normal((rows, cols))
    q, r = np.linalg.qr(g, mode="reduced")
    s = np.sign(np.diag(r))
    s[s == 0] = 1.0
    return q * s


def sigma_exp(r: int, scale: float) -> np.ndarray:
    """sigma_j = exp(-j/scale), j = 0..r-1."""
    return np.exp(-np.arange(r, dtype=np.float64) / scale)


def sigma_pow(r: int, power: float) -> np.ndarray:
    """sigma_j = (j+1)^(-power), j = 0..r-1."""
    return (np.arange(r, dtype=np.float64) + 1.0) ** (-power)


def sigma_logspace(r: int, lo_exp: float) -> np.ndarray:
    """r values logspaced from 1 down to 10^lo_exp (lo_exp < 0)."""
    return np.logspace(0.0, lo_exp, r)


def lowrank(m: int, n: int, sigma: np.ndarray, seed: int, rank: int | None = None,
            dtype=np.float64) -> np.ndarray:
    """A = U diag(sigma) V^T (m x n) with Haar U (m x r), V (n x r).

    ``rank`` (default min(m, n)) keeps only the leading ``rank`` terms; the leading
    columns of the Q factor of a Gaussian matrix depend only on its leading
    columns, so a truncated draw equals the leading part of the full one."""
    r = min(m, n) if rank is None else int(rank)
    sig = np.asarray(sigma, dtype=np.float64)[:r]
    u = haar_orthonormal(m, r, seed)
    v = haar_orthonormal(n, r, seed + 7919)
    a = (u * sig) @ v.T
    return np.ascontiguousarray(a.astype(dtype))


def lowrank_torch(m: int, n: int, sigma: np.ndarray, seed: int, device, rank: int | None = None):
    """The same construction as :func:`lowrank`, drawn with torch on ``device``
    (fast generation of the large workloads on the GPU). Returns float64.

    The draw differs from the NumPy one for the same seed; a test must take both
    sides' A from the same call."""
    import torch

    r = min(m, n) if rank is None else int(rank)
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    sig = torch.as_tensor(np.asarray(sigma, dtype=np.float64)[:r], device=device)

    def _haar(rows, cols):
        g = torch.randn(rows, cols, generator=gen, device=device, dtype=torch.float64)
        q, rr = torch.linalg.qr(g, mode="reduced")
        s = torch.sign(torch.diagonal(rr))
        s[s == 0] = 1.0
        return q * s

    u = _haar(m, r)
    v = _haar(n, r)
    return (u * sig) @ v.T


def noisy_lowrank_torch(m: int, n: int, sigma: np.ndarray, noise: float, seed: int, device):
    """:func:`lowrank_torch` plus i.i.d. N(0, noise^2) entries (the differentiable-ID
    workload: a decaying spectrum under a noise floor). Returns float64."""
    import torch

    a = lowrank_torch(m, n, sigma, seed, device)
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed) + 104729)
    return a + noise * torch.randn(m, n, generator=gen, device=device, dtype=torch.float64)


def noisy_lowrank_blocks_torch(nblk: int, m: int, n: int, power: float, noise: float, seed: int, device):
    """nblk blocks A_b = U_b diag((j+1)^-power) V_b^T + N(0, noise^2) (m x n each,
    Haar U_b, V_b from batched QRs of N(0,1) draws), as one float64 tensor of
    shape (nblk, m, n)."""
    import torch

    r = min(m, n)
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    sig = torch.as_tensor(sigma_pow(r, power), device=device)

    def _haar(rows):
        g = torch.randn(nblk, rows, r, generator=gen, device=device, dtype=torch.float64)
        q, rr = torch.linalg.qr(g, mode="reduced")
        s = torch.sign(torch.diagonal(rr, dim1=1, dim2=2))
        s[s == 0] = 1.0
        return q * s[:, None, :]

    u = _haar(m)
    v = _haar(n)
    a = (u * sig) @ v.transpose(1, 2)
    return a + noise * torch.randn(nblk, m, n, generator=gen, device=device, dtype=torch.float64)


def srht_draws(m: int, l: int, seed: int):
    """The random inputs of a subsampled randomized Hadamard sketch of an m-row
    matrix: ``rows`` (int32[l], distinct, uniform in [0, m') with m' the smallest
    power of two >= m) and ``signs`` (int8[m], +1 or -1 with equal probability)."""
    mp = 1
    while mp < m:
        mp *= 2
    if l > mp:
        raise ValueError("l exceeds the padded order")
    g = rng(seed)
    rows = g.choice(mp, size=l, replace=False).astype(np.int32)
    signs = (2 * g.integers(0, 2, size=m) - 1).astype(np.int8)
    return rows, signs


def gaussian(rows: int, cols: int, seed: int, dtype=np.float64) -> np.ndarray:
    """i.i.d. N(0,1) rows x cols matrix (row-major)."""
    return np.ascontiguousarray(rng(seed).standard_normal((rows, cols)).astype(dtype))


# ----------------------------------------------------------------------------
# Kernel blocks between well-separated point clusters.
# ----------------------------------------------------------------------------

def kernel_block_sizes(nblk: int, seed: int, lo: int = 64, hi: int = 512):
    """Block sizes (m_b, n_b), each uniform on the integers lo..hi inclusive."""
    g = rng(seed)
    ms = g.integers(lo, hi + 1, size=nblk)
    ns = g.integers(lo, hi + 1, size=nblk)
    return ms.astype(np.int64), ns.astype(np.int64)


def kernel_block(mb: int, nb: int, seed: int, block_id: int, dtype=np.float64) -> np.ndarray:
    """K_ij = 1/|x_i - y_j|; x uniform in [-1/2,1/2]^3, y uniform in the same cube
    shifted by (4, 0, 0). Points are redrawn per block from (seed, block_id)."""
    g = rng(seed * 1_000_003 + 17 * block_id + 1)
    x = g.random((mb, 3)) - 0.5
    y = g.random((nb, 3)) - 0.5
    y[:, 0] += 4.0
    d = np.sqrt(((x[:, None, :] - y[None, :, :]) ** 2).sum(axis=2))
    return np.ascontiguousarray((1.0 / d).astype(dtype))


def kernel_blocks_torch(nblk: int, seed: int, device, lo: int = 64, hi: int = 512):
    """The blocks of :func:`kernel_block` for block ids 0..nblk-1 with the sizes of
    :func:`kernel_block_sizes`: points drawn with NumPy exactly as there, the
    distances formed with torch on ``device`` in FP64 (same formula), returned as
    a list of contiguous FP32 device tensors."""
    import torch

    ms, ns = kernel_block_sizes(nblk, seed, lo, hi)
    out = []
    for b in range(nblk):
        g = rng(seed * 1_000_003 + 17 * b + 1)
        x = g.random((int(ms[b]), 3)) - 0.5
        y = g.random((int(ns[b]), 3)) - 0.5
        y[:, 0] += 4.0
        xt = torch.as_tensor(x, device=device)
        yt = torch.as_tensor(y, device=device)
        d = ((xt[:, None, :] - yt[None, :, :]) ** 2).sum(dim=2).sqrt()
        out.append((1.0 / d).to(torch.float32).contiguous())
    return out


# ----------------------------------------------------------------------------
# The five workload configurations (sizes and spectra).
# ----------------------------------------------------------------------------

@dataclass(frozen=True)
class Config:
    name: str
    m: int
    n: int
    k: int
    p: int          # oversampling; -1 means deterministic (no sketch)
    q: int          # orthonormalised power steps
    dtype: str
    sigma: str      # "exp:<scale>" | "pow:<power>"

    def spectrum(self) -> np.ndarray:
        kind, val = self.sigma.split(":")
        r = min(self.m, self.n)
        return sigma_exp(r, float(val)) if kind == "exp" else sigma_pow(r, float(val))

    def frobenius_floor(self) -> float:
        """Eckart-Young: min over rank-k B of |A-B|_F / |A|_F, from the spectrum."""
        s = self.spectrum()
        return float(math.sqrt((s[self.k:] ** 2).sum() / (s ** 2).sum()))


CONFIGS = {
    "det_fp64_2000x1000_k50": Config("det_fp64_2000x1000_k50", 2000, 1000, 50, -1, 0, "f64", "exp:10"),
    "rand_fp32_20000x10000_k200": Config("rand_fp32_20000x10000_k200", 20000, 10000, 200, 10, 1, "f32", "pow:2"),
    "mixed_50000x20000_k500": Config("mixed_50000x20000_k500", 50000, 20000, 500, 20, 1, "f32", "exp:80"),
    "diff_fp32_8192x4096_k128": Config("diff_fp32_8192x4096_k128", 8192, 4096, 128, 10, 0, "f32", "pow:1.5"),
}


def sparse_nonneg_csc(m: int, n: int, terms: int, xdens: float, ydens: float, decay: float, seed: int,
                      dtype=np.float64):
    """A sparse non-negative m x n matrix built from rank-1 terms, in compressed
    sparse column form: A = sum_t w_t x_t y_t^T with x_t (m) and y_t (n) sparse,
    their nonzeros uniform in (0, 1] at densities xdens and ydens, and weights
    w_t = exp(-t / decay). Returns (colptr int64[n+1], rowidx int32[nnz] sorted
    within each column, vals[nnz]) as NumPy arrays."""
    import scipy.sparse as sp
    g = rng(seed)
    X = sp.random(m, terms, density=xdens, format="csc", random_state=g,
                  data_rvs=lambda k: 1.0 - g.random(k))
    Y = sp.random(n, terms, density=ydens, format="csc", random_state=g,
                  data_rvs=lambda k: 1.0 - g.random(k))
    W = sp.diags(np.exp(-np.arange(terms, dtype=np.float64) / decay))
    A = (X @ W @ Y.T).tocsc()
    A.sort_indices()
    return (A.indptr.astype(np.int64), A.indices.astype(np.int32), A.data.astype(dtype))


def csc_to_dense(colptr, rowidx, vals, m: int, n: int) -> np.ndarray:
    """The dense m x n matrix of a compressed sparse column triple (repeated rows
    add up), by scipy."""
    import scipy.sparse as sp
    return sp.csc_matrix((np.asarray(vals, dtype=np.float64), np.asarray(rowidx), np.asarray(colptr)),
                         shape=(m, n)).toarray()
