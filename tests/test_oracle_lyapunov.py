"""Pins for the oracle's Lyapunov specialisation against LAPACK and closed forms."""
import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from oracle.closed_form import LaplaceSylvester
from oracle.lyapunov import spksm_lyapunov, tpksm_lyapunov
from workloads import make_config


def _dense(M):
    return M.to_scipy().toarray()


def test_exhaustion_equals_lapack_lyapunov():
    """d r = n with S = I: the projection space is R^n and X_d solves the Lyapunov equation
    exactly; compared with SciPy's solve_continuous_lyapunov (Bartels-Stewart in LAPACK)."""
    c = make_config("convdiff2d_1000", m=4, r=2)  # n = 16, nonsymmetric A
    n = c["n"]
    A = _dense(c["A"])
    X = sla.solve_continuous_lyapunov(A, c["C1"] @ c["C1"].T)
    I = sp.identity(n, format="csr")
    res = spksm_lyapunov(c["A"], c["C1"], k=3, maxit=n // 2, tol=0.0, p=1, S=I, trunc_tol=0.0)
    assert np.linalg.norm(res.X1 @ res.X2.T - X) < 1e-8 * np.linalg.norm(X)
    res_t = tpksm_lyapunov(c["A"], c["C1"], k=n, maxit=n // 2, tol=0.0, p=1, trunc_tol=0.0)
    assert np.linalg.norm(res_t.X1 @ res_t.X2.T - X) < 1e-8 * np.linalg.norm(X)


def test_solution_is_symmetric():
    """M_B = M_A and a symmetric right-hand side make the projected solution symmetric."""
    c = make_config("convdiff2d_1000", m=15, r=2)
    res = spksm_lyapunov(c["A"], c["C1"], k=2, maxit=12, tol=0.0, p=12, s=96, seed=5, trunc_tol=0.0)
    X = res.X1 @ res.X2.T
    assert np.linalg.norm(X - X.T) < 1e-10 * np.linalg.norm(X)


def test_laplacian_matches_closed_form():
    """A = L symmetric: L X + X L = C C^T has the sine-transform solution."""
    c = make_config("laplace2d_64", m=24)
    cf = LaplaceSylvester(24, c["C1"], c["C1"])
    res = spksm_lyapunov(c["A"], c["C1"], k=2, maxit=150, tol=1e-9, p=10, s=304, seed=3)
    assert res.status == "converged"
    assert cf.rel_error(res.X1, res.X2) < 1e-6


def test_shift_enters_both_sides():
    """(A + diag(sigma)) X + X (A + diag(sigma))^T = C C^T, checked at exhaustion."""
    c = make_config("reaction2d_500", m=4, r=1)  # n = 16
    n = c["n"]
    A = _dense(c["A"]) + np.diag(c["sigma"])
    X = sla.solve_continuous_lyapunov(A, c["C1"] @ c["C1"].T)
    res = spksm_lyapunov(c["A"], c["C1"], k=3, maxit=n, tol=0.0, p=1, S=sp.identity(n, format="csr"),
                         trunc_tol=0.0, sigma=c["sigma"])
    assert np.linalg.norm(res.X1 @ res.X2.T - X) < 1e-8 * np.linalg.norm(X)
