"""Pins for the oracle's Bartels-Stewart solver and the Laplacian closed form."""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import closed_form
from oracle.sylvester import bartels_stewart, kron_solve
from workloads import gaussian_factors, laplacian_2d


@pytest.mark.parametrize("m,q,seed", [(7, 5, 0), (30, 30, 1), (60, 45, 2)])
def test_bartels_stewart_matches_lapack(m, q, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    M = rng.standard_normal((m, m)) + 3 * np.eye(m)
    N = rng.standard_normal((q, q)) + 3 * np.eye(q)
    F = rng.standard_normal((m, q))
    Y = bartels_stewart(M, N, F)
    Yl = sla.solve_sylvester(M, N, F)  # LAPACK trsyl, an independent library routine
    assert np.linalg.norm(Y - Yl) <= 1e-12 * np.linalg.norm(Yl)
    assert np.linalg.norm(M @ Y + Y @ N - F) <= 1e-13 * np.linalg.norm(F) * (np.linalg.norm(M) + np.linalg.norm(N))


def test_bartels_stewart_indefinite_and_kron():
    """Eigenvalues on both sides of the imaginary axis: still the unique solution."""
    rng = np.random.Generator(np.random.PCG64(4))
    M = np.diag([-3.0, -1.0, 2.0, 5.0, 7.0]) + 0.3 * np.triu(rng.standard_normal((5, 5)), 1)
    M = sla.expm(0.1 * rng.standard_normal((5, 5))) @ M @ np.linalg.inv(sla.expm(0.1 * rng.standard_normal((5, 5))))
    N = rng.standard_normal((4, 4)) + 0.5 * np.eye(4)
    F = rng.standard_normal((5, 4))
    Y = bartels_stewart(M, N, F)
    assert np.allclose(Y, kron_solve(M, N, F), rtol=1e-11, atol=1e-12)


def test_dst_diagonalises_second_difference():
    m = 9
    Q = closed_form.dst_matrix(m)
    assert np.allclose(Q @ Q, np.eye(m), atol=1e-14)
    L = laplacian_2d(m).to_scipy().toarray()
    Q2 = np.kron(Q, Q)
    D = Q2 @ L @ Q2
    assert np.allclose(D, np.diag(closed_form.eigenvalues_2d(m)), atol=1e-9 * np.abs(D).max())


def test_closed_form_matches_dense_solve():
    m = 6
    L = laplacian_2d(m).to_scipy().toarray()
    C1, C2 = gaussian_factors(m * m, m * m, 2, 3)
    ref = bartels_stewart(L, L, C1 @ C2.T)
    cf = closed_form.LaplaceSylvester(m, C1, C2)
    X = cf.dense()
    assert np.linalg.norm(X - ref) <= 1e-12 * np.linalg.norm(ref)
    # rel_error of the exact solution in factored form is zero
    U, s, Vt = np.linalg.svd(ref)
    assert cf.rel_error(U * s, Vt.T) < 1e-12
