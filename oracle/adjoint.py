"""Gradients of ``L = tr(P1^T X P2)`` through the Sylvester solve, FP64.

``X`` solves ``(A0 + diag(sigma)) X + X B = C1 C2^T``.  With ``G = P1 P2^T`` and ``Lam``
solving the transposed equation ``A^T Lam + Lam B^T = G``:

* ``dL/dC1 = Lam C2``, ``dL/dC2 = Lam^T C1``;
* ``dL/dsigma_i = -sum_j Lam_ij X_ij``  (from ``dL = <Lam, dC - dA X>``);
* ``dL/dP1 = X P2``, ``dL/dP2 = X^T P1``.

``Lam ~ L1 L2^T`` comes from the same method run on ``(A^T, P1)`` and ``(B, P2)``, i.e.
``spksm(A^T, B^T, P1, P2)``.  Dense versions for tiny sizes use Bartels-Stewart on the
full matrices.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .spksm import as_operator, spksm
from .sylvester import bartels_stewart


def grads_from_factors(X1, X2, L1, L2, C1, C2, P1, P2) -> dict:
    dC1 = L1 @ (L2.T @ C2)
    dC2 = L2 @ (L1.T @ C1)
    dsigma = -np.sum((L1 @ (L2.T @ X2)) * X1, axis=1)
    dP1 = X1 @ (X2.T @ P2)
    dP2 = X2 @ (X1.T @ P1)
    loss = float(np.sum((P1.T @ X1) * (P2.T @ X2)))  # tr(P1^T X1 X2^T P2)
    return dict(loss=loss, dC1=dC1, dC2=dC2, dsigma=dsigma, dP1=dP1, dP2=dP2)


def solve_and_grad(A0, B, C1, C2, sigma, P1, P2, **params) -> dict:
    """Forward s-PKSM solve, adjoint s-PKSM solve and the gradients."""
    A0 = as_operator(A0)
    B = as_operator(B)
    fwd = spksm(A0, B, C1, C2, sigma=sigma, **params)
    At = A0.T.tocsr() if sp.issparse(A0) else A0.T
    Bt = B.T.tocsr() if sp.issparse(B) else B.T
    adj = spksm(At, Bt, P1, P2, sigma=sigma, **params)
    g = grads_from_factors(fwd.X1, fwd.X2, adj.X1, adj.X2, C1, C2, P1, P2)
    g["fwd"], g["adj"] = fwd, adj
    return g


def dense_grads(A0, B, C1, C2, sigma, P1, P2) -> dict:
    """Exact gradients from dense Bartels-Stewart solves (tiny sizes only)."""
    A = as_operator(A0)
    A = A.toarray() if sp.issparse(A) else np.asarray(A)
    if sigma is not None:
        A = A + np.diag(sigma)
    Bd = as_operator(B)
    Bd = Bd.toarray() if sp.issparse(Bd) else np.asarray(Bd)
    X = bartels_stewart(A, Bd, C1 @ C2.T)
    Lam = bartels_stewart(A.T, Bd.T, P1 @ P2.T)
    return dict(loss=float(np.sum(P1 * (X @ P2))), X=X, Lam=Lam, dC1=Lam @ C2, dC2=Lam.T @ C1,
                dsigma=-np.sum(Lam * X, axis=1), dP1=X @ P2, dP2=X.T @ P1)
