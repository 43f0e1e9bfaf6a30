"""Pins of the structured (subsampled randomized Hadamard) sketch oracle,
oracle/srht.py, the real counterpart of Section 5.2's eq. (def_srft)."""
import numpy as np
import pytest
import scipy.linalg

import synth
import oracle
from oracle import srht


@pytest.mark.parametrize("p", [0, 1, 2, 3, 5, 7])
def test_sign_formula_is_sylvester_hadamard(p):
    n = 2 ** p
    H = srht.hadamard_sign(np.arange(n)[:, None], np.arange(n)[None, :])
    assert np.array_equal(H, scipy.linalg.hadamard(n).astype(np.float64))


def test_fwht_of_unit_vectors_gives_hadamard_columns():
    n = 64
    Z = srht.fwht(np.eye(n))
    assert np.array_equal(Z, scipy.linalg.hadamard(n).astype(np.float64))


@pytest.mark.parametrize("m,n,l", [(64, 5, 16), (100, 7, 30), (1000, 9, 40), (129, 3, 128), (1, 4, 1)])
def test_fast_transform_equals_the_definition(m, n, l):
    A = synth.gaussian(m, n, seed=m + n + l)
    rows, signs = synth.srht_draws(m, l, seed=l + 3)
    Y_fast = srht.srht_sketch(A, rows, signs)
    Y_def = srht.srht_omega(m, rows, signs) @ A
    assert Y_fast.shape == (l, n)
    assert np.allclose(Y_fast, Y_def, rtol=0, atol=1e-12 * np.abs(A).sum(axis=0).max())


def test_rows_are_orthogonal_with_the_stated_scale():
    # m a power of two: Omega Omega^T = (m / l) I for distinct sampled rows
    m, l = 256, 40
    rows, signs = synth.srht_draws(m, l, seed=11)
    Om = srht.srht_omega(m, rows, signs)
    assert np.allclose(Om @ Om.T, (m / l) * np.eye(l), atol=1e-12)


def test_draws_are_distinct_and_in_range():
    rows, signs = synth.srht_draws(1000, 300, seed=5)
    assert len(set(rows.tolist())) == 300
    assert rows.min() >= 0 and rows.max() < 1024
    assert set(np.unique(signs).tolist()) <= {-1, 1}


def test_exact_rank_is_recovered_through_the_sketch():
    # an exactly rank-6 matrix: the ID on the structured sketch (l = 2k)
    # reconstructs it to rounding
    m, n, r = 300, 120, 6
    A = synth.lowrank(m, n, np.ones(r), seed=2, rank=r)
    rows, signs = synth.srht_draws(m, 2 * r, seed=9)
    res = oracle.id_col(A, r, omega=srht.srht_omega(m, rows, signs))
    assert res.k == r
    e = oracle.e_id(A, res.J, res.T)
    assert e < 1e-12
