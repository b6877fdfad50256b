"""Exact solution for ``A = B = L``, the 2D 5-point Dirichlet Laplacian (textbook, FP64).

With ``m`` interior nodes per direction and ``h = 1/(m+1)``, the 1D second difference
``(1/h^2) tridiag(-1, 2, -1)`` has orthonormal eigenvectors
``Q[a, j] = sqrt(2/(m+1)) sin((a+1)(j+1) pi/(m+1))`` (the DST-I matrix, symmetric and
its own inverse) and eigenvalues ``lam_j = (4/h^2) sin^2((j+1) pi / (2(m+1)))``.  The 2D
operator ``L = I kron T + T kron I`` is diagonalised by ``Q2 = Q kron Q`` with
eigenvalues ``mu = lam_x + lam_y``.  Hence ``L X + X L = C`` has the solution
``X = Q2 [ (Q2 C Q2) ./ (mu_i + mu_j) ] Q2``.

Only the transformed solution ``Xhat = (Q2 C Q2) ./ (mu_i + mu_j)`` is formed (``n x n``);
distances to a factored ``X1 X2^T`` are evaluated in the orthonormal ``Q2`` basis.
"""
from __future__ import annotations

import numpy as np


def dst_matrix(m: int) -> np.ndarray:
    j = np.arange(1, m + 1)
    return np.sqrt(2.0 / (m + 1)) * np.sin(np.outer(j, j) * np.pi / (m + 1))


def eigenvalues_2d(m: int) -> np.ndarray:
    """Eigenvalues of the 2D operator in the ``x``-fastest ordering (``mu[iy*m + ix]``)."""
    h = 1.0 / (m + 1)
    lam = 4.0 / h**2 * np.sin(np.arange(1, m + 1) * np.pi / (2 * (m + 1))) ** 2
    return (lam[:, None] + lam[None, :]).ravel()


def to_eigbasis(Qm: np.ndarray, X: np.ndarray) -> np.ndarray:
    """``Q2 X`` for ``X (m^2 x q)``; each column is an ``(iy, ix)`` grid reshaped."""
    m = Qm.shape[0]
    q = X.shape[1]
    G = X.T.reshape(q, m, m)                   # [col, iy, ix]
    G = np.einsum("ab,qbc,cd->qad", Qm, G, Qm)  # Q G Q (Q symmetric)
    return G.reshape(q, m * m).T


class LaplaceSylvester:
    """Exact solution of ``L X + X L = C1 C2^T`` on an ``m x m`` grid."""

    def __init__(self, m: int, C1: np.ndarray, C2: np.ndarray):
        self.m = m
        self.Q = dst_matrix(m)
        mu = eigenvalues_2d(m)
        P1 = to_eigbasis(self.Q, C1)
        P2 = to_eigbasis(self.Q, C2)
        self.Xhat = (P1 @ P2.T) / (mu[:, None] + mu[None, :])
        self.norm = float(np.linalg.norm(self.Xhat))

    def dense(self) -> np.ndarray:
        """The full ``n x n`` solution (small ``m`` only)."""
        Z = to_eigbasis(self.Q, self.Xhat)          # Q2 Xhat
        return to_eigbasis(self.Q, Z.T).T           # (Q2 (Q2 Xhat)^T)^T = Q2 Xhat Q2

    def rel_error(self, X1: np.ndarray, X2: np.ndarray) -> float:
        """``||X1 X2^T - X||_F / ||X||_F`` evaluated in the eigenbasis."""
        Z1 = to_eigbasis(self.Q, X1)
        Z2 = to_eigbasis(self.Q, X2)
        D = Z1 @ Z2.T - self.Xhat
        return float(np.linalg.norm(D)) / self.norm
