"""Pins of the oracle's comparison instruments at known, nonzero distances.

Every parity assertion goes through ``rel_distance`` (factored products) and the
closed-form checks through ``LaplaceSylvester.rel_error``; both are checked here against
dense evaluations and hand-computed values, so a wrong normalisation, a dropped factor or
a swapped argument fails.
"""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle.closed_form import LaplaceSylvester
from oracle.lowrank import product_fro, rel_distance, true_residual
from workloads import convdiff_2d_upwind, laplacian_2d


def _e(n, i):
    v = np.zeros((n, 1))
    v[i] = 1.0
    return v


def test_rel_distance_hand_computed_value():
    # Z = 3 e1 f1^T + 4 e2 f2^T, ||Z||_F = 5; X = Z + 12 e3 f4^T: distance 12 / 5
    n1, n2 = 7, 5
    Z1 = np.hstack([3 * _e(n1, 0), 4 * _e(n1, 1)])
    Z2 = np.hstack([_e(n2, 0), _e(n2, 1)])
    X1 = np.hstack([Z1, 12 * _e(n1, 2)])
    X2 = np.hstack([Z2, _e(n2, 3)])
    assert rel_distance(X1, X2, Z1, Z2) == pytest.approx(12 / 5, rel=1e-14)
    # normalised by the second argument: ||X||_F = 13, so the swapped distance is 12 / 13
    assert rel_distance(Z1, Z2, X1, X2) == pytest.approx(12 / 13, rel=1e-14)


def test_rel_distance_scaling_and_sign():
    rng = np.random.default_rng(0)
    Z1, Z2 = rng.standard_normal((30, 3)), rng.standard_normal((20, 3))
    assert rel_distance(2 * Z1, Z2, Z1, Z2) == pytest.approx(1.0, rel=1e-13)
    assert rel_distance(Z1, Z2, 2 * Z1, Z2) == pytest.approx(0.5, rel=1e-13)
    assert rel_distance(-Z1, Z2, Z1, Z2) == pytest.approx(2.0, rel=1e-13)
    # the factors are unique only up to X1 M, X2 M^{-T}: the distance sees the product only
    M = rng.standard_normal((3, 3)) + 3 * np.eye(3)
    assert rel_distance(Z1 @ M, Z2 @ np.linalg.inv(M).T, Z1, Z2) < 1e-13


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_rel_distance_matches_dense(seed):
    rng = np.random.default_rng(seed)
    n1, n2 = 25, 18
    X1, X2 = rng.standard_normal((n1, 4)), rng.standard_normal((n2, 4))
    Z1, Z2 = rng.standard_normal((n1, 2)), rng.standard_normal((n2, 2))
    dense = np.linalg.norm(X1 @ X2.T - Z1 @ Z2.T) / np.linalg.norm(Z1 @ Z2.T)
    assert dense > 0.5
    assert rel_distance(X1, X2, Z1, Z2) == pytest.approx(dense, rel=1e-12)
    # a small perturbation of known size: X = Z + eps u v^T with u, v unit and orthogonal to Z
    Q1, _ = np.linalg.qr(np.hstack([Z1, rng.standard_normal((n1, 1))]))
    Q2, _ = np.linalg.qr(np.hstack([Z2, rng.standard_normal((n2, 1))]))
    eps = 1e-7
    P1 = np.hstack([Z1, eps * Q1[:, 2:3]])
    P2 = np.hstack([Z2, Q2[:, 2:3]])
    assert rel_distance(P1, P2, Z1, Z2) == pytest.approx(eps / np.linalg.norm(Z1 @ Z2.T), rel=1e-6)


def test_product_fro_matches_dense():
    rng = np.random.default_rng(4)
    L, R = rng.standard_normal((40, 5)), rng.standard_normal((33, 5))
    assert product_fro(L, R) == pytest.approx(np.linalg.norm(L @ R.T), rel=1e-13)
    # wide factors (more columns than rows) too
    L, R = rng.standard_normal((6, 9)), rng.standard_normal((7, 9))
    assert product_fro(L, R) == pytest.approx(np.linalg.norm(L @ R.T), rel=1e-13)


@pytest.mark.parametrize("with_sigma", [False, True])
def test_true_residual_matches_dense_at_nonzero_residual(with_sigma):
    rng = np.random.default_rng(5)
    A = convdiff_2d_upwind(5, 1e-2, (1.0, 0.5)).to_scipy().toarray()
    B = convdiff_2d_upwind(5, 1e-2, (-0.3, 1.0)).to_scipy().toarray()
    n = A.shape[0]
    C1, C2 = rng.standard_normal((n, 2)), rng.standard_normal((n, 2))
    X1, X2 = rng.standard_normal((n, 3)), rng.standard_normal((n, 3))
    sigma = rng.uniform(0, 1, n) if with_sigma else None
    Ad = A + (np.diag(sigma) if with_sigma else 0)
    X = X1 @ X2.T
    dense = np.linalg.norm(Ad @ X + X @ B - C1 @ C2.T) / np.linalg.norm(C1 @ C2.T)
    assert dense > 1.0
    assert true_residual(A, B, C1, C2, X1, X2, sigma=sigma) == pytest.approx(dense, rel=1e-12)
    # the exact solution (LAPACK's Bartels-Stewart) has a residual at rounding level
    Xs = sla.solve_sylvester(Ad, B, C1 @ C2.T)
    U, s, Vt = np.linalg.svd(Xs)
    assert true_residual(A, B, C1, C2, U * s, Vt.T, sigma=sigma) < 1e-12


def test_closed_form_rel_error_at_known_distance():
    m = 4
    L = laplacian_2d(m).to_scipy().toarray()
    n = L.shape[0]
    rng = np.random.default_rng(6)
    C1, C2 = rng.standard_normal((n, 2)), rng.standard_normal((n, 2))
    cf = LaplaceSylvester(m, C1, C2)
    X = sla.solve_sylvester(L, L, C1 @ C2.T)  # independent of the sine transform
    assert cf.norm == pytest.approx(np.linalg.norm(X), rel=1e-12)
    U, s, Vt = np.linalg.svd(X)
    X1, X2 = U * s, Vt.T
    assert cf.rel_error(X1, X2) < 1e-12
    assert cf.rel_error(2 * X1, X2) == pytest.approx(1.0, rel=1e-12)
    # X + eps u v^T with unit u, v: distance eps / ||X||_F
    eps = 1e-3
    u, v = _e(n, 3), _e(n, 7)
    Y1, Y2 = np.hstack([X1, eps * u]), np.hstack([X2, v])
    assert cf.rel_error(Y1, Y2) == pytest.approx(eps / np.linalg.norm(X), rel=1e-8)
    # and against a dense evaluation of an arbitrary factored guess
    G1, G2 = rng.standard_normal((n, 3)) * 1e-3, rng.standard_normal((n, 3))
    dense = np.linalg.norm(G1 @ G2.T - X) / np.linalg.norm(X)
    assert cf.rel_error(G1, G2) == pytest.approx(dense, rel=1e-12)
