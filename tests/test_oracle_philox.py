"""Pins for the oracle's Philox4x32-10 generator and the Gaussian sketch matrix."""
import os

import numpy as np
import scipy.stats

from oracle import philox

HERE = os.path.dirname(os.path.abspath(__file__))


def _kat():
    rows = []
    with open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                w = [int(x, 16) for x in line.split()]
                rows.append((w[:4], w[4:6], w[6:10]))
    return rows


def test_known_answer_vectors():
    kat = _kat()
    assert len(kat) == 3
    for ctr, key, out in kat:
        got = philox.philox4x32_10(np.array([ctr], dtype=np.uint64), np.array(key, dtype=np.uint64))
        assert [int(v) for v in got[0]] == out


def test_gaussian_is_standard_normal():
    z = philox.gaussian_omega(200, 1000, seed=123).ravel()
    assert abs(z.mean()) < 0.01 and abs(z.std() - 1.0) < 0.01
    assert scipy.stats.kstest(z, "norm").pvalue > 1e-3


def test_elementwise_definition_and_streams():
    rows, cols = 3, 7
    om = philox.gaussian_omega(rows, cols, seed=99, stream=2)
    # recompute entry (r, i) from its own counter
    for r in range(rows):
        for i in range(cols):
            f = r * cols + i
            g = f // 4
            w = philox.philox4x32_10(np.array([[g, 0, 2, 0]], dtype=np.uint64),
                                     np.array([99, 0], dtype=np.uint64))[0].astype(np.float64)
            pair = (f % 4) // 2
            u1 = (w[2 * pair] + 1.0) / 2.0 ** 32
            u2 = w[2 * pair + 1] / 2.0 ** 32
            rho = np.sqrt(-2.0 * np.log(u1))
            want = rho * (np.cos if f % 2 == 0 else np.sin)(2 * np.pi * u2)
            assert om[r, i] == want
    other = philox.gaussian_omega(rows, cols, seed=99, stream=3)
    assert not np.array_equal(om, other)
