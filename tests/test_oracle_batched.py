"""Pins of the oracle's adaptive-rank batched column ID (oracle/batched.py).

* exactly rank-r blocks: the rank found is r, the reconstruction exact, and the
  sketch width doubles exactly when r exceeds l_0 - p;
* the rank cap: a block of rank above l_cap - p stops at l_cap - p, flagged;
* the tolerance rank is the smallest j whose residual, recomputed from an
  independent QR of the first j pivot columns of Y, is within tol |Y|_F;
* on the kernel blocks of the batched workload the sketched rank tracks the
  deterministic tolerance rank of the block itself, and the true ID error stays
  of the order of the tolerance.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import synth
from oracle import batched


def _omega(lcap, m, seed=1):
    return synth.gaussian(lcap, m, seed=seed)


def _rank_r(m, n, r, seed):
    return synth.lowrank(m, n, synth.sigma_pow(r, 1.0), seed=seed, rank=r)


def test_exact_rank_below_first_width():
    A = _rank_r(120, 90, 11, seed=1)
    res = batched.id_col_adaptive(A, _omega(56, 120), p=8, tol=1e-6, kmax=48)
    assert res.met and res.l == 32 and res.id.k == 11
    assert oracle.e_id(A, res.id.J, res.id.T) <= 1e-12


def test_width_doubles_when_rank_exceeds_first_cap():
    # l_0 = 32, p = 8: 24 steps are not enough for rank 30, l doubles to l_cap = 56
    A = _rank_r(150, 100, 30, seed=2)
    res = batched.id_col_adaptive(A, _omega(56, 150), p=8, tol=1e-6, kmax=48)
    assert res.met and res.l == 56 and res.id.k == 30
    assert oracle.e_id(A, res.id.J, res.id.T) <= 1e-11


def test_rank_cap_flags_and_stops():
    A = _rank_r(140, 120, 60, seed=3)
    res = batched.id_col_adaptive(A, _omega(48, 140), p=8, tol=1e-6, kmax=40)
    assert not res.met and res.l == 48 and res.id.k == 40


def test_tolerance_rank_is_smallest_by_independent_residuals():
    g = synth.rng(4)
    A = synth.lowrank(100, 80, synth.sigma_exp(80, 3.0), seed=4)
    om = _omega(40, 100)
    tol = 1e-4
    res = batched.id_col_adaptive(A, om, p=6, tol=tol, kmax=34)
    assert res.met
    Y = om[:res.l] @ A
    yf = np.linalg.norm(Y)

    def resid(j):
        if j == 0:
            return yf
        Q, _ = np.linalg.qr(Y[:, res.id.J[:j]])
        return np.linalg.norm(Y - Q @ (Q.T @ Y))

    k = res.id.k
    assert resid(k) <= tol * yf * (1 + 1e-9)
    assert resid(k - 1) > tol * yf
    del g


def test_fixed_rank_mode_is_the_sketched_id():
    A = synth.lowrank(90, 70, synth.sigma_exp(70, 4.0), seed=5)
    om = _omega(20, 90)
    res = batched.id_col_adaptive(A, om, p=8, k=12)
    ref = oracle.id_col(A, 12, omega=om[:20])
    assert res.l == 20 and np.array_equal(res.id.J, ref.J) and np.allclose(res.id.T, ref.T, atol=1e-12)


@pytest.mark.parametrize("b", [0, 1, 2, 3])
def test_kernel_blocks_track_deterministic_rank(b):
    ms, ns = synth.kernel_block_sizes(4, seed=7)
    A = synth.kernel_block(int(ms[b]), int(ns[b]), seed=7, block_id=b)
    om = _omega(64, int(ms[b]), seed=8)
    tol = 1e-6
    res = batched.id_col_adaptive(A, om, p=8, tol=tol, kmax=56)
    det = oracle.cpqr(A, 64, tol=tol)
    assert res.met
    assert abs(res.id.k - det.k_out) <= 3
    assert oracle.e_id(A, res.id.J, res.id.T) <= 20 * tol
