"""The Lyapunov specialisation ``A X + X A^T = C C^T`` of Algorithms 1 and 2, plain FP64.
Test infrastructure only: the GPU library never calls it.

With ``B = A^T`` and ``C2 = C1 = C`` the second Krylov space ``K_d(B^T, C2)`` of the
Sylvester methods is ``K_d(A, C)`` itself (the setting of the paper's Sec. 4), so one basis
serves both sides; for s-PKSM both sides then use the same embedding ``S`` (the one the
Sylvester solve would draw for ``S_U``), which makes the projected matrices equal,
``M_B = M_A``, and the projected solution symmetric.  This module states exactly that
reading by calling the two-space oracles with ``B = (A + diag(sigma))^T``, ``C2 = C`` and
``S_V = S_U``.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import sketch as _sketch
from .spksm import as_operator, spksm
from .tpksm import tpksm


def _shifted(A, sigma):
    A = as_operator(A)
    if sigma is None:
        return A
    D = sp.diags(np.asarray(sigma, dtype=np.float64)) if sp.issparse(A) else np.diag(sigma)
    return (A + D).tocsr() if sp.issparse(A) else A + D


def spksm_lyapunov(A, C, *, k: int, maxit: int, tol: float, p: int = 1, s: int | None = None, zeta: int = 8,
                   seed: int = 0, sketch: str = "sparse_sign", S=None, trunc_tol: float = 1e-12,
                   recover: str = "stored", sigma=None, keep: bool = False, orth: str = "euclidean"):
    """s-PKSM for ``(A + diag(sigma)) X + X (A + diag(sigma))^T = C C^T``."""
    As = _shifted(A, sigma)
    C = np.asarray(C, dtype=np.float64)
    n, r = C.shape
    if s is None:
        s = 2 * maxit * r
    if S is None:
        S = _sketch.make(sketch, n, s, zeta, _sketch.space_seeds(seed)[0])
    return spksm(As, As.T, C, C, k=k, maxit=maxit, tol=tol, p=p, s=s, S_U=S, S_V=S, trunc_tol=trunc_tol,
                 recover=recover, keep=keep, orth=orth)


def tpksm_lyapunov(A, C, *, k: int, maxit: int, tol: float, p: int = 1, trunc_tol: float = 1e-12,
                   recover: str = "stored", sigma=None, keep: bool = False):
    """t-PKSM (Algorithm 2) for the same Lyapunov equation."""
    As = _shifted(A, sigma)
    C = np.asarray(C, dtype=np.float64)
    return tpksm(As, As.T, C, C, k=k, maxit=maxit, tol=tol, p=p, trunc_tol=trunc_tol, recover=recover, keep=keep)
