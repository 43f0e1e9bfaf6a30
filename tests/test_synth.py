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
