"""Norms of low-rank products without forming them (FP64).

The factored solution ``X = X1 X2^T`` is unique only up to ``X1 M, X2 M^{-T}``, so every
comparison here acts on products.  ``||L R^T||_F`` for tall ``L``, ``R`` is evaluated as
``||R_L R_R^T||_F`` from thin QR factorisations of ``L`` and ``R``.
"""
from __future__ import annotations

import numpy as np

from .spksm import as_operator


def product_fro(L: np.ndarray, R: np.ndarray) -> float:
    """``||L R^T||_F`` for ``L (n1 x q)``, ``R (n2 x q)``."""
    _, RL = np.linalg.qr(L, mode="reduced")
    _, RR = np.linalg.qr(R, mode="reduced")
    return float(np.linalg.norm(RL @ RR.T))


def rel_distance(X1, X2, Z1, Z2) -> float:
    """``||X1 X2^T - Z1 Z2^T||_F / ||Z1 Z2^T||_F``."""
    num = product_fro(np.hstack([X1, -Z1]), np.hstack([X2, Z2]))
    return num / product_fro(Z1, Z2)


def true_residual(A, B, C1, C2, X1, X2, sigma=None) -> float:
    """Relative residual ``||A X + X B - C1 C2^T||_F / ||C1 C2^T||_F`` for ``X = X1 X2^T``.

    ``A X + X B - C1 C2^T = [A X1, X1, -C1] [X2, B^T X2, C2]^T``.
    """
    A = as_operator(A)
    B = as_operator(B)
    AX1 = A @ X1
    if sigma is not None:
        AX1 = AX1 + np.asarray(sigma)[:, None] * X1
    L = np.hstack([AX1, X1, -C1])
    R = np.hstack([X2, B.T @ X2, C2])
    return product_fro(L, R) / product_fro(C1, C2)
