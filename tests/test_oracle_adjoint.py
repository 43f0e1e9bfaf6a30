"""Pins of the oracle's reconstruction-loss gradient (oracle/adjoint.py).

The gradient formulas are checked against derivatives computed without them:
complex-step differentiation of the loss (Squire & Trapp 1998; the loss is
analytic because every product uses plain transposes), central differences of
a loss that solves its least-squares problem with a library routine, and the
deterministic closed form where the path through T vanishes.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import synth
from oracle import adjoint


def _case(m, n, k, l, seed, noise=0.0):
    rng = synth.rng(seed)
    A = synth.lowrank(m, n, synth.sigma_pow(min(m, n), 1.5), seed=seed)
    if noise:
        A = A + noise * rng.standard_normal((m, n))
    om = None if l is None else synth.gaussian(l, m, seed=seed + 1)
    Y = A if om is None else om @ A
    J = oracle.cpqr(Y, k).J
    return A, om, J


def _loss_lstsq(A, J, k, om):
    # the same loss with T from LAPACK least squares (a different route)
    J1, J2 = J[:k], J[k:]
    Y = A if om is None else om @ A
    T = np.linalg.lstsq(Y[:, J1], Y[:, J2], rcond=None)[0]
    E = A[:, J2] - A[:, J1] @ T
    return float(np.sum(E * E))


@pytest.mark.parametrize("sketch", [False, True])
def test_every_entry_against_complex_step(sketch):
    m, n, k = 7, 6, 2
    A, om, J = _case(m, n, k, 4 if sketch else None, seed=11, noise=1e-2)
    G = adjoint.recon_grad(A, J, k, om)
    h = 1e-30
    num = np.zeros_like(A)
    for i in range(m):
        for j in range(n):
            Ac = A.astype(np.complex128)
            Ac[i, j] += 1j * h
            num[i, j] = adjoint.recon_loss(Ac, J, k, om).imag / h
    assert np.allclose(G, num, rtol=1e-10, atol=1e-13 * np.abs(num).max())


@pytest.mark.parametrize("sketch", [False, True])
def test_directional_derivative_complex_step(sketch):
    m, n, k = 60, 40, 6
    A, om, J = _case(m, n, k, 10 if sketch else None, seed=5, noise=1e-3)
    D = synth.rng(99).standard_normal((m, n))
    G = adjoint.recon_grad(A, J, k, om)
    h = 1e-30
    d_cs = adjoint.recon_loss(A + 1j * h * D, J, k, om).imag / h
    assert abs(np.sum(G * D) - d_cs) <= 1e-9 * abs(d_cs)


def test_directional_derivative_central_difference_library_lstsq():
    m, n, k = 60, 40, 6
    A, om, J = _case(m, n, k, 10, seed=8, noise=1e-3)
    D = synth.rng(3).standard_normal((m, n))
    G = adjoint.recon_grad(A, J, k, om)
    eps = 1e-6
    d_fd = (_loss_lstsq(A + eps * D, J, k, om) - _loss_lstsq(A - eps * D, J, k, om)) / (2 * eps)
    assert abs(np.sum(G * D) - d_fd) <= 1e-6 * max(abs(d_fd), 1e-12)


def test_deterministic_path_through_t_vanishes():
    # without a sketch T solves the least-squares problem for A itself, so
    # C^T E = 0 and the gradient is 2E on J2 and -2 E T^T on J1
    m, n, k = 50, 30, 5
    A, om, J = _case(m, n, k, None, seed=2, noise=1e-3)
    J1, J2 = J[:k], J[k:]
    C = A[:, J1]
    T = np.linalg.lstsq(C, A[:, J2], rcond=None)[0]
    E = A[:, J2] - C @ T
    ref = np.zeros_like(A)
    ref[:, J2] = 2 * E
    ref[:, J1] = -2 * E @ T.T
    G = adjoint.recon_grad(A, J, k, None)
    assert np.allclose(G, ref, rtol=0, atol=1e-10 * np.abs(ref).max())


def test_loss_matches_e_id():
    # the loss is (e_ID |A|_F)^2 of the column ID (Section 2.3)
    m, n, k = 40, 30, 4
    A, om, J = _case(m, n, k, 9, seed=4, noise=1e-3)
    J1, J2 = J[:k], J[k:]
    Y = om @ A
    T = np.linalg.lstsq(Y[:, J1], Y[:, J2], rcond=None)[0]
    e = oracle.e_id(A, J, T)
    assert np.isclose(adjoint.recon_loss(A, J, k, om), (e * np.linalg.norm(A)) ** 2, rtol=1e-10)
