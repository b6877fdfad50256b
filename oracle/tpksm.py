"""Algorithm 2 of the paper (t-PKSM, the truncated Arnoldi method of appendix A), plain
FP64 NumPy/SciPy, step by step.  Test infrastructure only: the GPU library never calls it.

The two truncated block Arnoldi recurrences are those of Algorithm 1 (space U on ``A``
from ``C1``, space V on ``B^T`` from ``C2``; modified block Gram-Schmidt against the last
``k`` blocks, oldest first, one pass; thin QR with a positive diagonal), with no
embedding.  Every ``p`` steps (and at ``maxit``) the projected equation is the one on the
truncated block Hessenberg matrices themselves,

    H_d Y + Y G_d^T = E_1 beta_1 beta_2^T E_1^T,

with ``beta_1``, ``beta_2`` the R factors of ``C1``, ``C2``, and the residual estimate of
Algorithm 2 is

    rho = sqrt(d r) (||Y E_d g_{d+1,d}^T||_F + ||h_{d+1,d} E_d^T Y||_F),

compared with ``tol * ||beta_1 beta_2^T||_F`` (the same relative reading as for
Algorithm 1).  The factors are ``X1 = U_d Y1``, ``X2 = V_d Y2`` from the truncated SVD of
``Y`` (no whitening), from the stored blocks or by the two-pass replay.  Breakdown
handling is that of the s-PKSM oracle.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .spksm import BREAKDOWN_REL_DIAG, BREAKDOWN_REL_NORM, Result, as_operator, qr_pos
from .sylvester import bartels_stewart


class TruncatedSpace:
    """One truncated block Arnoldi recurrence (no embedding)."""

    def __init__(self, op, k: int, r: int, maxit: int, keep_all: bool):
        self.op, self.k, self.r, self.maxit, self.keep_all = op, k, r, maxit, keep_all
        self.H = np.zeros(((maxit + 1) * r, maxit * r))
        self.blocks = {}
        self.ell = None
        self.broken = False

    def init(self, C: np.ndarray) -> None:
        U1, self.ell = qr_pos(C)
        self.blocks[1] = U1

    def step(self, d: int) -> None:
        r = self.r
        Ut = self.op(self.blocks[d])
        nrm_op = np.linalg.norm(Ut)
        for i in range(max(1, d - self.k + 1), d + 1):
            h = self.blocks[i].T @ Ut
            Ut = Ut - self.blocks[i] @ h
            self.H[(i - 1) * r:i * r, (d - 1) * r:d * r] = h
        Unew, hsub = qr_pos(Ut)
        dg = np.abs(np.diag(hsub))
        if (np.linalg.norm(Ut) < BREAKDOWN_REL_NORM * nrm_op
                or dg.min() < BREAKDOWN_REL_DIAG * max(np.abs(hsub).max(), np.finfo(float).tiny)):
            self.broken = True
            hsub = np.zeros((r, r))
            Unew = np.zeros_like(Ut)
        self.H[d * r:(d + 1) * r, (d - 1) * r:d * r] = hsub
        self.blocks[d + 1] = Unew
        if not self.keep_all:
            for j in list(self.blocks):
                if j < d + 2 - self.k:
                    del self.blocks[j]

    def replay(self, C: np.ndarray, d: int, W: np.ndarray) -> np.ndarray:
        """Second pass: regenerate U_1 .. U_d from the stored H and accumulate U_j W[j]."""
        r = self.r
        U = {1: sla.solve_triangular(self.ell.T, C.T, lower=True).T}
        X = U[1] @ W[:r]
        for j in range(1, d):
            Ut = self.op(U[j])
            for i in range(max(1, j - self.k + 1), j + 1):
                Ut = Ut - U[i] @ self.H[(i - 1) * r:i * r, (j - 1) * r:j * r]
            hsub = self.H[j * r:(j + 1) * r, (j - 1) * r:j * r]
            U[j + 1] = sla.solve_triangular(hsub.T, Ut.T, lower=True).T
            X = X + U[j + 1] @ W[j * r:(j + 1) * r]
            for i in list(U):
                if i < j + 2 - self.k:
                    del U[i]
        return X


def tpksm(A, B, C1, C2, *, k: int, maxit: int, tol: float, p: int = 1, trunc_tol: float = 1e-12,
          recover: str = "stored", sigma=None, keep: bool = False) -> Result:
    """Solve ``A X + X B = C1 C2^T`` with t-PKSM; returns low-rank ``X ~ X1 X2^T``."""
    A = as_operator(A)
    B = as_operator(B)
    C1 = np.asarray(C1, dtype=np.float64)
    C2 = np.asarray(C2, dtype=np.float64)
    r = C1.shape[1]
    if C2.shape[1] != r:
        raise ValueError("C1 and C2 must have the same number of columns")
    sig = None if sigma is None else np.asarray(sigma, dtype=np.float64)[:, None]
    BT = B.T

    def op_u(X):
        Y = A @ X
        return Y if sig is None else Y + sig * X

    keep_all = recover == "stored" or keep
    U = TruncatedSpace(op_u, k, r, maxit, keep_all)
    V = TruncatedSpace(lambda X: BT @ X, k, r, maxit, keep_all)
    U.init(C1)
    V.init(C2)
    F11 = U.ell @ V.ell.T  # beta_1 beta_2^T
    rhs = float(np.linalg.norm(F11))

    history, status, Y, d = [], "maxit", None, 0
    for d in range(1, maxit + 1):
        U.step(d)
        V.step(d)
        broken = U.broken or V.broken
        if d % p == 0 or d == maxit or broken:
            m = d * r
            Hd, Gd = U.H[:m, :m], V.H[:m, :m]
            F = np.zeros((m, m))
            F[:r, :r] = F11
            Y = bartels_stewart(Hd, Gd.T, F)
            h_sub = U.H[m:m + r, m - r:m]
            g_sub = V.H[m:m + r, m - r:m]
            rho = np.sqrt(m) * (np.linalg.norm(Y[:, m - r:] @ g_sub.T) + np.linalg.norm(h_sub @ Y[m - r:, :]))
            history.append((d, rho / rhs))
            if broken:
                status = "breakdown"
                break
            if rho <= tol * rhs:
                status = "converged"
                break

    Phi, sv, PsiT = np.linalg.svd(Y)
    ell = int(np.sum(sv > trunc_tol * sv[0])) if trunc_tol > 0 else int(np.sum(sv > 0))
    ell = max(ell, 1)
    sq = np.sqrt(sv[:ell])
    W1 = Phi[:, :ell] * sq
    W2 = PsiT[:ell].T * sq
    if recover == "stored":
        X1 = np.hstack([U.blocks[j] for j in range(1, d + 1)]) @ W1
        X2 = np.hstack([V.blocks[j] for j in range(1, d + 1)]) @ W2
    elif recover == "two_pass":
        X1 = U.replay(C1, d, W1)
        X2 = V.replay(C2, d, W2)
    else:
        raise ValueError(recover)
    return Result(X1=X1, X2=X2, d=d, status=status, history=history, rhs_norm=rhs, ell=ell,
                  Y=Y if keep else None)
