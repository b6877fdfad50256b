"""Algorithm 1 of the paper (s-PKSM), plain FP64 NumPy/SciPy, step by step.

Notation follows the paper: the two Krylov spaces are built on ``A`` (space U, start
block ``C1``) and on ``B^T`` (space V, start block ``C2``); ``H``/``G`` are the banded
block Hessenberg matrices of the truncated Arnoldi relations (eqn:arnoldi_tr);
``S_U U = Q_U T_U`` is the QR factorisation of the sketched basis of Prop. 2.1.

Readings taken where the paper is terse, garbled or silent (each one is exercised by
a test):

* Initialisation of Algorithm 1: ``S_V`` sketches ``C2`` (the algorithm prints ``S_U``),
  ``T_{U,1}`` is the R factor of ``S_U U_1`` and ``beta_1 = T_{U,1} l`` is the R factor
  of ``S_U C1`` (the algorithm prints ``T_{U,1} = beta_1``, which contradicts Prop. 2.1's
  definition of ``T`` unless ``l = I``).
* Orthogonalisation: modified block Gram-Schmidt against the last ``k`` blocks, oldest
  first, one pass (Algorithm 1, inner loop); the window includes ``U_d``.
* Thin QR: the unique factorisation with a positive diagonal in ``R`` (Householder
  with a sign fix).
* Sketched QR update (Prop. 2.1): classical Gram-Schmidt of ``S_U U_{d+1}`` against
  ``Q_U`` with one re-orthogonalisation pass, then a thin QR of the remainder.
* Projected matrices: ``M_A = T_{U,d+1} H_d_bar T_{U,d}^{-1}`` (the closed form of
  eqn:Hhat_Ghat); its top ``dr`` rows are ``Hhat_d + Hhat E_d^T`` and its last block row
  is ``[0 ... 0, tau_{d+1} h_{d+1,d} tau_d^{-1}]``.  The residual estimate uses this
  *whitened* subdiagonal block; only then does it equal ``||S_U R S_V^T||_F``
  (eq:resnorm_sk prints the unwhitened ``h_{d+1,d}``).
* Stop test: ``rho <= tol * ||beta_1 beta_2^T||_F`` (relative; equal to the paper's
  absolute test when ``||C1 C2^T||_F = 1`` as in its experiments up to the embedding
  distortion), checked when ``d`` is a multiple of ``p`` and always at ``d = maxit``.
* Breakdown (not discussed in the paper): if the orthogonalised block is negligible
  (``||U~||_F < 1e-12 ||A U_d||_F``) or its R factor is numerically singular
  (``min diag < 1e-14 max |R|``), the space is exhausted; its subdiagonal block is set
  to zero, a final projected solve is done and the status is ``breakdown``.
* Low-rank factors (the closing factorisation and retrieval of Algorithm 1): the SVD ``Y = Phi Sigma Psi^T`` is
  truncated at ``sigma_i > trunc_tol * sigma_1``; ``X1 = U_d T_U^{-1} Phi_l Sigma_l^(1/2)``
  and ``X2 = V_d T_V^{-1} Psi_l Sigma_l^(1/2)``.
* Two-pass recovery (Sec. 5): ``U_1 = C1 l^{-1}`` and
  ``U_{j+1} = (A U_j - sum_{i=max(1,j-k+1)}^{j} U_i h_{i,j}) h_{j+1,j}^{-1}`` replayed with
  the stored ``H``; the stored-basis recovery is the reference.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from . import sketch as _sketch
from .sylvester import bartels_stewart

BREAKDOWN_REL_NORM = 1e-12
BREAKDOWN_REL_DIAG = 1e-14


def qr_pos(X: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """Thin Householder QR with the signs fixed so that ``diag(R) >= 0``."""
    Q, R = np.linalg.qr(X, mode="reduced")
    sgn = np.sign(np.diag(R))
    sgn[sgn == 0] = 1.0
    return Q * sgn[None, :], sgn[:, None] * R


def as_operator(M):
    """Accept a SciPy sparse matrix, a dense array or a ``workloads.CSR``."""
    if hasattr(M, "to_scipy"):
        return M.to_scipy()
    if sp.issparse(M):
        return M.tocsr()
    return np.asarray(M, dtype=np.float64)


@dataclass
class Space:
    """One truncated block Arnoldi recurrence with its sketched QR factorisation."""

    op: object                 # callable X -> Op X
    S: object                  # s x n embedding (supports S @ X)
    k: int
    r: int
    maxit: int
    keep_all: bool
    blocks: dict = field(default_factory=dict)   # j (1-based) -> n x r block
    H: np.ndarray = None       # ((maxit+1) r) x (maxit r), banded block Hessenberg
    T: np.ndarray = None       # ((maxit+1) r) square, upper triangular
    Q: np.ndarray = None       # s x ((maxit+1) r), orthonormal columns
    ell: np.ndarray = None     # R factor of the start block
    beta: np.ndarray = None    # R factor of S C
    broken: bool = False
    orth: str = "euclidean"    # 'euclidean' (Algorithm 1) or 'sketched' (inner products of S x)
    sblocks: dict = field(default_factory=dict)  # j -> S U_j (orth = 'sketched')

    def init(self, C: np.ndarray) -> None:
        r, m1 = self.r, (self.maxit + 1) * self.r
        if self.orth == "sketched":  # U_1 ell = C with S U_1 orthonormal: ell = R factor of S C
            _, self.ell = qr_pos(self.S @ C)
            U1 = sla.solve_triangular(self.ell.T, C.T, lower=True).T
        else:
            U1, self.ell = qr_pos(C)
        W = self.S @ U1
        s = W.shape[0]
        self.H = np.zeros((m1, self.maxit * r))
        self.T = np.zeros((m1, m1))
        self.Q = np.zeros((s, m1))
        q, t = qr_pos(W)
        self.Q[:, :r] = q
        self.T[:r, :r] = t
        self.beta = t @ self.ell
        self.blocks[1] = U1
        self.sblocks[1] = W

    def step(self, d: int) -> None:
        """Block step ``d``: SpMM, truncated MGS, thin QR, sketched QR update."""
        if self.orth == "sketched":
            self.step_sketched(d)
            return
        r = self.r
        Ut = self.op(self.blocks[d])
        nrm_op = np.linalg.norm(Ut)
        for i in range(max(1, d - self.k + 1), d + 1):
            Ui = self.blocks[i]
            h = Ui.T @ Ut
            Ut = Ut - Ui @ h
            self.H[(i - 1) * r:i * r, (d - 1) * r:d * r] = h
        Unew, hsub = qr_pos(Ut)
        dg = np.abs(np.diag(hsub))
        if (np.linalg.norm(Ut) < BREAKDOWN_REL_NORM * nrm_op
                or dg.min() < BREAKDOWN_REL_DIAG * max(np.abs(hsub).max(), np.finfo(float).tiny)):
            self.broken = True
            hsub = np.zeros((r, r))
            Unew = np.zeros_like(Ut)
            TH, tau, q = np.zeros((d * r, r)), np.eye(r), np.zeros((self.Q.shape[0], r))
        else:
            w = self.S @ Unew
            Qd = self.Q[:, :d * r]
            c1 = Qd.T @ w
            w = w - Qd @ c1
            c2 = Qd.T @ w
            w = w - Qd @ c2
            q, tau = qr_pos(w)
            TH = c1 + c2
        self.H[d * r:(d + 1) * r, (d - 1) * r:d * r] = hsub
        self.T[:d * r, d * r:(d + 1) * r] = TH
        self.T[d * r:(d + 1) * r, d * r:(d + 1) * r] = tau
        self.Q[:, d * r:(d + 1) * r] = q
        self.blocks[d + 1] = Unew
        if not self.keep_all:
            for j in list(self.blocks):
                if j < d + 2 - self.k:
                    del self.blocks[j]

    def step_sketched(self, d: int) -> None:
        """Block step ``d`` with the sketched inner product <x, y>_S = (S x)^T (S y) in the
        truncated Gram-Schmidt and in the thin QR (the variant the paper's appendix A
        mentions): ``S U~`` is formed once and updated linearly in the sketch space, the
        orthogonalisation coefficients and the QR factor come from it, and ``U~`` itself is
        updated once with all coefficients; then ``S U_{d+1} = (S U~) R^{-1}`` feeds the
        sketched QR update of Prop. 2.1 as before."""
        r = self.r
        Ut = self.op(self.blocks[d])
        SUt = self.S @ Ut
        nrm_op = np.linalg.norm(SUt)
        coef = []
        for i in range(max(1, d - self.k + 1), d + 1):
            h = self.sblocks[i].T @ SUt
            SUt = SUt - self.sblocks[i] @ h
            self.H[(i - 1) * r:i * r, (d - 1) * r:d * r] = h
            coef.append((i, h))
        for i, h in coef:
            Ut = Ut - self.blocks[i] @ h
        _, hsub = qr_pos(SUt)  # R factor in the sketched norm
        dg = np.abs(np.diag(hsub))
        if (np.linalg.norm(SUt) < BREAKDOWN_REL_NORM * nrm_op
                or dg.min() < BREAKDOWN_REL_DIAG * max(np.abs(hsub).max(), np.finfo(float).tiny)):
            self.broken = True
            hsub = np.zeros((r, r))
            Unew = np.zeros_like(Ut)
            w = np.zeros_like(SUt)
            TH, tau, q = np.zeros((d * r, r)), np.eye(r), np.zeros((self.Q.shape[0], r))
        else:
            Unew = sla.solve_triangular(hsub.T, Ut.T, lower=True).T    # U~ R^{-1}
            w = sla.solve_triangular(hsub.T, SUt.T, lower=True).T      # S U_{d+1}
            Qd = self.Q[:, :d * r]
            c1 = Qd.T @ w
            w2 = w - Qd @ c1
            c2 = Qd.T @ w2
            w2 = w2 - Qd @ c2
            q, tau = qr_pos(w2)
            TH = c1 + c2
        self.H[d * r:(d + 1) * r, (d - 1) * r:d * r] = hsub
        self.T[:d * r, d * r:(d + 1) * r] = TH
        self.T[d * r:(d + 1) * r, d * r:(d + 1) * r] = tau
        self.Q[:, d * r:(d + 1) * r] = q
        self.blocks[d + 1] = Unew
        self.sblocks[d + 1] = w
        for store in (self.blocks, self.sblocks):
            if store is self.sblocks or not self.keep_all:
                for j in list(store):
                    if j < d + 2 - self.k:
                        del store[j]

    def projected(self, d: int) -> tuple[np.ndarray, np.ndarray]:
        """``M = T_{d+1} H_d_bar T_d^{-1}``: top ``dr`` rows and the last block row's last block."""
        r, m = self.r, d * self.r
        Z = self.T[:m + r, :m + r] @ self.H[:m + r, :m]
        Mbar = sla.solve_triangular(self.T[:m, :m], Z.T, trans="T", lower=False).T
        return Mbar[:m], Mbar[m:, m - r:]

    def replay(self, C: np.ndarray, op, d: int, W: np.ndarray) -> np.ndarray:
        """Two-pass recovery: regenerate ``U_1..U_d`` from ``H`` and accumulate ``U_j W[j]``."""
        r = self.r
        U = {1: sla.solve_triangular(self.ell.T, C.T, lower=True).T}  # C l^{-1}
        X = U[1] @ W[:r]
        for j in range(1, d):
            Ut = op(U[j])
            for i in range(max(1, j - self.k + 1), j + 1):
                Ut = Ut - U[i] @ self.H[(i - 1) * r:i * r, (j - 1) * r:j * r]
            hsub = self.H[j * r:(j + 1) * r, (j - 1) * r:j * r]
            U[j + 1] = sla.solve_triangular(hsub.T, Ut.T, lower=True).T  # Ut hsub^{-1}
            X = X + U[j + 1] @ W[j * r:(j + 1) * r]
            for i in list(U):
                if i < j + 2 - self.k:
                    del U[i]
        return X


@dataclass
class Result:
    X1: np.ndarray
    X2: np.ndarray
    d: int
    status: str                    # 'converged' | 'maxit' | 'breakdown'
    history: list                  # [(d, rho / ||beta1 beta2^T||_F)]
    rhs_norm: float
    ell: int
    Y: np.ndarray = None
    U: Space = None
    V: Space = None


def spksm(A, B, C1, C2, *, k: int, maxit: int, tol: float, p: int = 1, s: int | None = None,
          zeta: int = 8, seed: int = 0, sketch: str = "sparse_sign", S_U=None, S_V=None,
          trunc_tol: float = 1e-12, recover: str = "stored", sigma=None,
          keep: bool = False, orth: str = "euclidean") -> Result:
    """Solve ``A X + X B = C1 C2^T`` with s-PKSM; returns low-rank ``X ~ X1 X2^T``.

    ``orth = 'sketched'`` orthogonalises the truncated bases with the sketched inner product
    (see ``Space.step_sketched``); the projected problem and everything after it are
    unchanged.

    ``sigma`` (optional, length ``n1``) adds ``diag(sigma)`` to ``A``.  ``S_U``/``S_V``
    override the embeddings (e.g. the identity for the ``S = I`` special case).
    """
    A = as_operator(A)
    B = as_operator(B)
    C1 = np.asarray(C1, dtype=np.float64)
    C2 = np.asarray(C2, dtype=np.float64)
    n1, r = C1.shape
    n2 = C2.shape[0]
    if C2.shape[1] != r:
        raise ValueError("C1 and C2 must have the same number of columns")
    if s is None:
        s = 2 * maxit * r
    seed_u, seed_v = _sketch.space_seeds(seed)
    if S_U is None:
        S_U = _sketch.make(sketch, n1, s, zeta, seed_u)
    if S_V is None:
        S_V = _sketch.make(sketch, n2, s, zeta, seed_v)
    sig = None if sigma is None else np.asarray(sigma, dtype=np.float64)[:, None]
    BT = B.T

    def op_u(X):
        Y = A @ X
        return Y if sig is None else Y + sig * X

    def op_v(X):
        return BT @ X

    keep_all = recover == "stored" or keep
    if orth not in ("euclidean", "sketched"):
        raise ValueError(orth)
    U = Space(op_u, S_U, k, r, maxit, keep_all, orth=orth)
    V = Space(op_v, S_V, k, r, maxit, keep_all, orth=orth)
    U.init(C1)
    V.init(C2)
    F11 = U.beta @ V.beta.T
    rhs = float(np.linalg.norm(F11))

    history, status, Y, d = [], "maxit", None, 0
    for d in range(1, maxit + 1):
        U.step(d)
        V.step(d)
        broken = U.broken or V.broken
        if d % p == 0 or d == maxit or broken:
            m = d * r
            MA, hhat = U.projected(d)
            MB, ghat = V.projected(d)
            F = np.zeros((m, m))
            F[:r, :r] = F11
            Y = bartels_stewart(MA, MB.T, F)
            rho = np.sqrt(np.linalg.norm(hhat @ Y[m - r:, :]) ** 2 + np.linalg.norm(Y[:, m - r:] @ ghat.T) ** 2)
            history.append((d, rho / rhs))
            if broken:
                status = "breakdown"
                break
            if rho <= tol * rhs:
                status = "converged"
                break

    m = d * r
    Phi, sv, PsiT = np.linalg.svd(Y)
    ell = int(np.sum(sv > trunc_tol * sv[0])) if trunc_tol > 0 else int(np.sum(sv > 0))
    ell = max(ell, 1)
    sq = np.sqrt(sv[:ell])
    W1 = sla.solve_triangular(U.T[:m, :m], Phi[:, :ell] * sq, lower=False)
    W2 = sla.solve_triangular(V.T[:m, :m], PsiT[:ell].T * sq, lower=False)
    if recover == "stored":
        X1 = np.hstack([U.blocks[j] for j in range(1, d + 1)]) @ W1
        X2 = np.hstack([V.blocks[j] for j in range(1, d + 1)]) @ W2
    elif recover == "two_pass":
        X1 = U.replay(C1, op_u, d, W1)
        X2 = V.replay(C2, op_v, d, W2)
    else:
        raise ValueError(recover)
    return Result(X1=X1, X2=X2, d=d, status=status, history=history, rhs_norm=rhs, ell=ell,
                  Y=Y if keep else None, U=U if keep else None, V=V if keep else None)
