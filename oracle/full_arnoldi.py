"""Full block Arnoldi Galerkin solution (Sec. 2.1 and eqn:full), a test reference only.

Builds orthonormal bases of ``K_d(A, C1)`` and ``K_d(B^T, C2)`` by block Gram-Schmidt
against *all* previous blocks, applied twice (so the basis is orthonormal to rounding),
projects explicitly (``H = U^T A U``, ``G = V^T B^T V``) and solves the Galerkin equation
``H Y + Y G^T = U^T C1 C2^T V`` with SciPy's LAPACK-based ``solve_sylvester``.  The exact
residual norm is evaluated from the factored residual.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .spksm import as_operator


def _basis(op, C, d):
    n, r = C.shape
    U = np.zeros((n, d * r))
    Q, _ = np.linalg.qr(C)
    U[:, :r] = Q
    for j in range(1, d):
        W = op(U[:, (j - 1) * r:j * r])
        for _ in range(2):
            W = W - U[:, :j * r] @ (U[:, :j * r].T @ W)
        Q, _ = np.linalg.qr(W)
        U[:, j * r:(j + 1) * r] = Q
    return U


def full_arnoldi_galerkin(A, B, C1, C2, d, sigma=None):
    """Return ``(X1, X2)`` with ``X = U_d Y V_d^T`` of the full Arnoldi Galerkin method."""
    A = as_operator(A)
    B = as_operator(B)
    sig = None if sigma is None else np.asarray(sigma)[:, None]

    def op_a(X):
        Y = A @ X
        return Y if sig is None else Y + sig * X

    U = _basis(op_a, C1, d)
    V = _basis(lambda X: B.T @ X, C2, d)
    H = U.T @ op_a(U)
    G = V.T @ (B.T @ V)
    F = (U.T @ C1) @ (V.T @ C2).T
    Y = sla.solve_sylvester(H, G.T, F)
    return U @ Y, V
