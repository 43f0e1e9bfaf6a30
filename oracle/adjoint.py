"""Gradient of the column-ID reconstruction loss with the skeleton frozen.

THIS MODULE IS TEST INFRASTRUCTURE (see the package header).

Loss (the column ID of Section 2.3 / Algorithm 1, sketched as in Section 5.1):

    Y = Omega A  (or Y = A without a sketch),   J = [J1 J2] frozen,
    T = argmin_X |Y(:,J1) X - Y(:,J2)|_F        (= S11^{-1} S12, eq. (S11T=S12)),
    E = A(:,J2) - A(:,J1) T,                     L = |E|_F^2.

The derivative follows the chain rule through the least-squares solution
(Golub & Pereyra 1973 for the derivative of a pseudo-inverse solution):

    dL = 2 <E, dA(:,J2) - dA(:,J1) T - A(:,J1) dT>
    dT = (Y1^T Y1)^{-1} [ dY1^T Rres + Y1^T (dY2 - dY1 T) ],   Rres = Y2 - Y1 T

so with Tbar = -2 A(:,J1)^T E and M = (Y1^T Y1)^{-1} Tbar:

    Abar(:,J2) = 2 E,   Abar(:,J1) = -2 E T^T,
    Ybar2 = Y1 M,       Ybar1 = Rres M^T - Y1 M T^T,
    Abar += Omega^T Ybar       (Ybar(:,J1) = Ybar1, Ybar(:,J2) = Ybar2).

Every product uses plain transposes (no conjugation), so the loss is an
analytic function of A and the formulas hold for complex A as well; the tests
use that for a complex-step check. Omega is not differentiated.
"""
from __future__ import annotations

import numpy as np


def _split(J, k):
    J = np.asarray(J)
    return J[:k], J[k:]


def interp_lstsq(Y1: np.ndarray, Y2: np.ndarray) -> np.ndarray:
    """T = (Y1^T Y1)^{-1} Y1^T Y2 by the normal equations (transpose, not conjugate),
    usable for complex arguments; for real data it is the least-squares T."""
    return np.linalg.solve(Y1.T @ Y1, Y1.T @ Y2)


def recon_loss(A: np.ndarray, J, k: int, omega: np.ndarray | None = None) -> float:
    """L = |A(:,J2) - A(:,J1) T|_F^2 with T from the (sketched) skeleton columns.
    For complex A returns sum(E*E) (no conjugate), the analytic continuation."""
    J1, J2 = _split(J, k)
    Y = A if omega is None else omega @ A
    T = interp_lstsq(Y[:, J1], Y[:, J2])
    E = A[:, J2] - A[:, J1] @ T
    return np.sum(E * E)


def recon_grad(A: np.ndarray, J, k: int, omega: np.ndarray | None = None) -> np.ndarray:
    """dL/dA for recon_loss (J frozen, Omega fixed), by the formulas above."""
    J1, J2 = _split(J, k)
    Y = A if omega is None else omega @ A
    Y1, Y2 = Y[:, J1], Y[:, J2]
    G = Y1.T @ Y1
    T = np.linalg.solve(G, Y1.T @ Y2)
    C = A[:, J1]
    E = A[:, J2] - C @ T
    Abar = np.zeros_like(A)
    Abar[:, J2] += 2.0 * E
    Abar[:, J1] += -2.0 * E @ T.T
    Tbar = -2.0 * C.T @ E
    M = np.linalg.solve(G, Tbar)
    Rres = Y2 - Y1 @ T
    Ybar = np.zeros_like(Y)
    Ybar[:, J2] = Y1 @ M
    Ybar[:, J1] = Rres @ M.T - Y1 @ M @ T.T
    if omega is None:
        Abar += Ybar
    else:
        Abar += omega.T @ Ybar
    return Abar
