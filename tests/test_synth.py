"""The seeded input generators: determinism and the advertised structure."""
import numpy as np

import synth


def test_seeded_and_orthonormal():
    a = synth.haar_orthonormal(50, 20, 1)
    b = synth.haar_orthonormal(50, 20, 1)
    assert np.array_equal(a, b)
    assert np.abs(a.T @ a - np.eye(20)).max() <= 1e-13


def test_lowrank_has_prescribed_spectrum():
    sig = synth.sigma_pow(30, 2.0)
    A = synth.lowrank(60, 30, sig, seed=2)
    s = np.linalg.svd(A, compute_uv=False)
    assert np.abs(s - sig).max() <= 1e-13


def test_truncated_draw_is_leading_part():
    sig = synth.sigma_exp(40, 3.0)
    full = synth.haar_orthonormal(60, 40, 3)
    part = synth.haar_orthonormal(60, 40, 3)[:, :10]
    assert np.array_equal(full[:, :10], part)


def test_kernel_blocks():
    ms, ns = synth.kernel_block_sizes(100, 4)
    assert ms.min() >= 64 and ms.max() <= 512 and ns.min() >= 64 and ns.max() <= 512
    K = synth.kernel_block(70, 90, 4, 5)
    assert K.shape == (70, 90)
    assert 0.17 < K.min() and K.max() < 0.34
    assert np.array_equal(K, synth.kernel_block(70, 90, 4, 5))


def test_config_floors():
    c = synth.CONFIGS["det_fp64_2000x1000_k50"]
    s = c.spectrum()
    assert abs(s[50] / s[0] - np.exp(-5.0)) < 1e-15
    c2 = synth.CONFIGS["rand_fp32_20000x10000_k200"]
    assert abs(c2.frobenius_floor() - 1.955e-4) < 2e-6


def test_sparse_nonneg_csc_structure_and_densify():
    """The sparse generator gives a valid compressed-sparse-column triple
    (nondecreasing pointers, sorted in-range rows, non-negative values), its rank
    is at most the number of terms, and csc_to_dense agrees with an entry-by-
    entry loop, repeated rows adding up."""
    m, n, terms = 500, 40, 12
    cp, ri, v = synth.sparse_nonneg_csc(m, n, terms, 0.05, 0.4, 4.0, seed=3)
    assert cp[0] == 0 and cp[-1] == ri.size == v.size and np.all(np.diff(cp) >= 0)
    assert ri.min() >= 0 and ri.max() < m and v.min() > 0
    for j in range(n):
        assert np.all(np.diff(ri[cp[j]:cp[j + 1]]) > 0)
    D = synth.csc_to_dense(cp, ri, v, m, n)
    assert np.linalg.matrix_rank(D) <= terms
    # an irregular triple with a repeated row, against a loop
    cp2 = np.array([0, 3, 3, 5], np.int64)
    ri2 = np.array([4, 1, 4, 0, 2], np.int32)
    v2 = np.array([1.0, 2.0, 3.0, -1.0, 0.5])
    E = np.zeros((6, 3))
    for j in range(3):
        for q in range(cp2[j], cp2[j + 1]):
            E[ri2[q], j] += v2[q]
    assert np.array_equal(synth.csc_to_dense(cp2, ri2, v2, 6, 3), E)
    assert E[4, 0] == 4.0
    a = synth.sparse_nonneg_csc(m, n, terms, 0.05, 0.4, 4.0, seed=3)
    assert all(np.array_equal(x, y) for x, y in zip(a, (cp, ri, v)))
