"""Pins for the oracle's Algorithm 1 (s-PKSM) against what the paper and mathematics fix.

None of these re-types the oracle's own formulas: each compares it with an independent
construction (full Arnoldi with LAPACK's Sylvester solver, dense Bartels-Stewart on the
full equation, an explicitly formed sketched residual, the sine-transform closed form)
or with an exact identity the paper states.
"""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

from oracle import sketch
from oracle.closed_form import LaplaceSylvester
from oracle.full_arnoldi import full_arnoldi_galerkin
from oracle.lowrank import rel_distance, true_residual
from oracle.spksm import spksm
from oracle.sylvester import bartels_stewart
from workloads import make_config


def _small(name, m, r=None):
    return make_config(name, m=m, r=r)


def _dense(M):
    return M.to_scipy().toarray()


@pytest.mark.parametrize("k", [1, 2, 4])
def test_identity_sketch_equals_full_arnoldi(k):
    """S = I: the whitened basis is Euclidean-orthonormal, so s-PKSM is the full Arnoldi
    Galerkin method for any k (the S^T S-Galerkin condition of Sec. 3 with S = I) and
    rho is the exact residual norm (eq:resnorm_sk)."""
    c = _small("convdiff2d_1000", 11, r=2)
    n, d = c["n"], 7
    I = sp.identity(n, format="csr")
    res = spksm(c["A"], c["B"], c["C1"], c["C2"], k=k, maxit=d, tol=0.0, p=1, S_U=I, S_V=I, trunc_tol=0.0)
    F1, F2 = full_arnoldi_galerkin(c["A"], c["B"], c["C1"], c["C2"], d)
    assert rel_distance(res.X1, res.X2, F1, F2) < 1e-11
    tr = true_residual(c["A"], c["B"], c["C1"], c["C2"], res.X1, res.X2)
    assert abs(res.history[-1][1] / tr - 1) < 1e-10


def test_krylov_exhaustion_gives_exact_solution():
    """d r = n with S = I: the projection space is all of R^n and X_d = X."""
    c = _small("convdiff2d_1000", 4, r=2)  # n = 16
    n = c["n"]
    I = sp.identity(n, format="csr")
    res = spksm(c["A"], c["B"], c["C1"], c["C2"], k=3, maxit=n // 2, tol=0.0, p=1, S_U=I, S_V=I, trunc_tol=0.0)
    X = bartels_stewart(_dense(c["A"]), _dense(c["B"]), c["C1"] @ c["C2"].T)
    assert np.linalg.norm(res.X1 @ res.X2.T - X) < 1e-8 * np.linalg.norm(X)


def _explicit_sketched_residual(c, res, S_U, S_V):
    X = res.X1 @ res.X2.T
    A, B = _dense(c["A"]), _dense(c["B"])
    R = A @ X + X @ B - c["C1"] @ c["C2"].T
    return np.linalg.norm(S_U @ R @ S_V.T)


@pytest.mark.parametrize("kind", ["gaussian", "sparse_sign"])
def test_rho_equals_sketched_residual_norm(kind):
    """eq:resnorm_sk as an identity: rho = ||S_U R_d S_V^T||_F with R_d formed densely.

    This fixes the reading of the subdiagonal block in the estimate: it must be the
    whitened tau_{d+1} h_{d+1,d} tau_d^{-1}."""
    c = _small("convdiff2d_1000", 8, r=2)  # n = 64
    n, s, d = c["n"], 48, 6
    su, sv = sketch.space_seeds(7)
    S_U = sketch.make(kind, n, s, 8, su)
    S_V = sketch.make(kind, n, s, 8, sv)
    S_Ud = S_U.toarray() if sp.issparse(S_U) else S_U
    S_Vd = S_V.toarray() if sp.issparse(S_V) else S_V
    res = spksm(c["A"], c["B"], c["C1"], c["C2"], k=2, maxit=d, tol=0.0, p=1, S_U=S_Ud, S_V=S_Vd,
                trunc_tol=0.0, keep=True)
    rho = res.history[-1][1] * res.rhs_norm
    ref = _explicit_sketched_residual(c, res, S_Ud, S_Vd)
    assert abs(rho / ref - 1) < 1e-9
    # planted reading: the unwhitened h_{d+1,d} (as printed) does not satisfy the identity
    r, m = 2, d * 2
    h_raw = res.U.H[m:m + r, m - r:m]
    g_raw = res.V.H[m:m + r, m - r:m]
    Y = res.Y
    rho_raw = np.sqrt(np.linalg.norm(h_raw @ Y[m - r:]) ** 2 + np.linalg.norm(Y[:, m - r:] @ g_raw.T) ** 2)
    assert abs(rho_raw / ref - 1) > 1e-3


def test_init_reading_beta_is_R_of_sketched_rhs():
    """Algorithm 1's init: beta_1 = T_{U,1} l equals the R factor of S_U C1."""
    c = _small("convdiff2d_1000", 8, r=3)
    res = spksm(c["A"], c["B"], c["C1"], c["C2"], k=2, maxit=2, tol=0.0, p=1, s=48, seed=5, keep=True)
    S_U = sketch.make("sparse_sign", c["n"], 48, 8, sketch.space_seeds(5)[0])
    _, R = np.linalg.qr(S_U @ c["C1"])
    R = np.sign(np.diag(R))[:, None] * R
    assert np.allclose(res.U.beta, R, rtol=1e-12, atol=1e-14)


def test_structural_invariants():
    """Truncated Arnoldi relation (eqn:arnoldi_tr), local orthogonality, and the sketched
    QR S_U U_{d+1} = Q T of Prop. 2.1 with orthonormal Q and positive-diagonal T."""
    c = _small("convdiff2d_1000", 10, r=2)
    d, r, k = 9, 2, 3
    res = spksm(c["A"], c["B"], c["C1"], c["C2"], k=k, maxit=d, tol=0.0, p=100, s=96, seed=3, keep=True)
    U = res.U
    Ud = np.hstack([U.blocks[j] for j in range(1, d + 2)])
    A = c["A"].to_scipy()
    lhs = A @ Ud[:, :d * r]
    rhs = Ud @ U.H[:(d + 1) * r, :d * r]
    assert np.linalg.norm(lhs - rhs) < 1e-13 * sla.norm(A.toarray(), 2) * np.sqrt(d)
    for j in range(1, d + 2):
        Uj = U.blocks[j]
        assert np.allclose(Uj.T @ Uj, np.eye(r), atol=1e-13)
        for i in range(max(1, j - k), j):
            assert np.abs(U.blocks[i].T @ Uj).max() < 1e-12
    S = sketch.make("sparse_sign", c["n"], 96, 8, sketch.space_seeds(3)[0])
    m1 = (d + 1) * r
    Q, T = U.Q[:, :m1], U.T[:m1, :m1]
    assert np.allclose(Q.T @ Q, np.eye(m1), atol=1e-13)
    assert np.allclose(np.tril(T, -1), 0) and np.all(np.diag(T) > 0)
    assert np.linalg.norm(S @ Ud - Q @ T) < 1e-13 * np.linalg.norm(T)


def test_incremental_Hhat_update_corrected():
    """The block update of Sec. 5 for Hhat_{d+1} equals T H T^{-1} once the last term of
    Hhat_new carries tau_{d+1}^{-1}; as printed (tau_d^{-1}) it does not."""
    c = _small("convdiff2d_1000", 9, r=2)
    d, r = 5, 2
    res = spksm(c["A"], c["B"], c["C1"], c["C2"], k=2, maxit=d + 1, tol=0.0, p=100, s=64, seed=11, keep=True)
    T, H = res.U.T, res.U.H
    m, m1 = d * r, (d + 1) * r
    Td, TH, tau1, taud = T[:m, :m], T[:m, m:m1], T[m:m1, m:m1], T[m - r:m, m - r:m]
    Hd, hsub = H[:m, :m], H[m:m1, m - r:m]
    Hcol, hdiag = H[:m, m:m1], H[m:m1, m:m1]
    inv = np.linalg.inv
    Hhat_d = Td @ Hd @ inv(Td)
    E = np.zeros((m, r))
    E[m - r:] = np.eye(r)
    top = Hhat_d + TH @ hsub @ inv(taud) @ E.T
    new_fixed = -top @ TH @ inv(tau1) + Td @ Hcol @ inv(tau1) + TH @ hdiag @ inv(tau1)
    new_printed = -top @ TH @ inv(tau1) + Td @ Hcol @ inv(tau1) + TH @ hdiag @ inv(taud)
    bottom_left = tau1 @ hsub @ inv(taud) @ E.T
    bottom_right = tau1 @ (-hsub @ inv(taud) @ E.T @ TH + hdiag) @ inv(tau1)
    closed = T[:m1, :m1] @ H[:m1, :m1] @ inv(T[:m1, :m1])
    inc = np.block([[top, new_fixed], [bottom_left, bottom_right]])
    scale = np.linalg.norm(closed)
    assert np.linalg.norm(inc - closed) < 1e-10 * scale
    assert np.linalg.norm(np.block([[top, new_printed], [bottom_left, bottom_right]]) - closed) > 1e-6 * scale


def test_two_pass_equals_stored():
    c = _small("laplace2d_64", 16)
    kw = dict(k=2, maxit=40, tol=1e-9, p=5, s=160, seed=1)
    a = spksm(c["A"], c["B"], c["C1"], c["C2"], recover="stored", **kw)
    b = spksm(c["A"], c["B"], c["C1"], c["C2"], recover="two_pass", **kw)
    assert a.d == b.d
    assert rel_distance(b.X1, b.X2, a.X1, a.X2) < 1e-11


def test_scale_invariance_of_the_embedding():
    """X_d does not change when S is multiplied by a scalar (T, beta and Y absorb it)."""
    c = _small("convdiff2d_1000", 8, r=2)
    n, s = c["n"], 48
    su, sv = sketch.space_seeds(2)
    S_U = sketch.make("sparse_sign", n, s, 8, su)
    S_V = sketch.make("sparse_sign", n, s, 8, sv)
    kw = dict(k=2, maxit=8, tol=0.0, p=1, trunc_tol=0.0)
    a = spksm(c["A"], c["B"], c["C1"], c["C2"], S_U=S_U, S_V=S_V, **kw)
    b = spksm(c["A"], c["B"], c["C1"], c["C2"], S_U=3.0 * S_U, S_V=0.5 * S_V, **kw)
    assert rel_distance(b.X1, b.X2, a.X1, a.X2) < 1e-10
    assert abs(a.history[-1][1] - b.history[-1][1]) < 1e-10 * a.history[-1][1]


def test_laplace_converges_to_closed_form():
    c = _small("laplace2d_64", 32)
    res = spksm(c["A"], c["B"], c["C1"], c["C2"], k=2, maxit=200, tol=1e-9, p=10, s=400, seed=1001)
    assert res.status == "converged"
    cf = LaplaceSylvester(32, c["C1"], c["C2"])
    tr = true_residual(c["A"], c["B"], c["C1"], c["C2"], res.X1, res.X2)
    assert tr < 5e-9
    assert cf.rel_error(res.X1, res.X2) < 1e-6


@pytest.mark.parametrize("name,m", [("convdiff2d_1000", 10), ("aniso3d_100", 5), ("reaction2d_500", 10),
                                    ("lognormal2d_2000", 10)])
def test_each_workload_family_matches_dense_solve(name, m):
    c = _small(name, m, r=2)
    A = _dense(c["A"])
    if c["sigma"] is not None:
        A = A + np.diag(c["sigma"])
    X = bartels_stewart(A, _dense(c["B"]), c["C1"] @ c["C2"].T)
    res = spksm(c["A"], c["B"], c["C1"], c["C2"], sigma=c["sigma"], k=2, maxit=45, tol=1e-10, p=1,
                s=200, seed=c["sketch_seed"])
    err = np.linalg.norm(res.X1 @ res.X2.T - X) / np.linalg.norm(X)
    assert err < 1e-6, (res.status, res.d, err)


def test_breakdown_on_invariant_subspace():
    """A diagonal A with 3 distinct eigenvalues: K_d(A, c) stops growing at d = 3."""
    n = 30
    A = sp.diags(np.tile([1.0, 2.0, 4.0], n // 3)).tocsr()
    rng = np.random.Generator(np.random.PCG64(1))
    B = sp.csr_matrix(np.diag(np.linspace(1, 3, n)) + 0.1 * np.triu(rng.standard_normal((n, n)), 1))
    C1 = rng.standard_normal((n, 1))
    C2 = rng.standard_normal((n, 1))
    I = sp.identity(n, format="csr")
    res = spksm(A, B, C1, C2, k=2, maxit=10, tol=0.0, p=5, S_U=I, S_V=I)
    assert res.status == "breakdown" and res.d == 3
    tr = true_residual(A, B, C1, C2, res.X1, res.X2)
    assert abs(res.history[-1][1] / tr - 1) < 1e-8
