"""Small dense Sylvester equations ``M Y + Y N = F`` by Bartels-Stewart, FP64.

The paper solves every projected equation with the Bartels-Stewart algorithm
(Sec. 6, where MATLAB's ``lyap`` is named).  Written out:

1. complex Schur forms ``M = Qa Ra Qa^*`` and ``N = Qb Rb Qb^*`` (``Ra``, ``Rb`` upper
   triangular);
2. ``G = Qa^* F Qb``;
3. the triangular equation ``Ra Z + Z Rb = G`` column by column: column ``j`` solves
   ``(Ra + Rb[j,j] I) z_j = g_j - sum_{i<j} Rb[i,j] z_i``, an upper triangular system;
4. ``Y = Qa Z Qb^*`` (real part for real data).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def bartels_stewart(M: np.ndarray, N: np.ndarray, F: np.ndarray) -> np.ndarray:
    """Solve ``M Y + Y N = F`` for square ``M (m x m)``, ``N (q x q)``, ``F (m x q)``."""
    M = np.asarray(M, dtype=np.float64)
    N = np.asarray(N, dtype=np.float64)
    F = np.asarray(F, dtype=np.float64)
    m, q = F.shape
    Ra, Qa = sla.schur(M, output="complex")
    Rb, Qb = sla.schur(N, output="complex")
    G = Qa.conj().T @ F @ Qb
    Z = np.zeros((m, q), dtype=np.complex128)
    eye = np.eye(m)
    for j in range(q):
        rhs = G[:, j] - Z[:, :j] @ Rb[:j, j]
        Z[:, j] = sla.solve_triangular(Ra + Rb[j, j] * eye, rhs, lower=False)
    Y = Qa @ Z @ Qb.conj().T
    return Y.real.copy()


def kron_solve(M: np.ndarray, N: np.ndarray, F: np.ndarray) -> np.ndarray:
    """Brute force: solve ``(I kron M + N^T kron I) vec(Y) = vec(F)`` densely (tiny sizes only)."""
    m, q = F.shape
    K = np.kron(np.eye(q), M) + np.kron(N.T, np.eye(m))
    y = np.linalg.solve(K, F.reshape(-1, order="F"))
    return y.reshape((m, q), order="F")
