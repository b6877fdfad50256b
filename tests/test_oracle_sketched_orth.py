"""Pins for the sketched-inner-product orthogonalisation (the variant of the truncated
Arnoldi steps that appendix A mentions): the sketched Galerkin projection of Algorithm 1
depends only on the Krylov spaces and the embeddings, not on the basis, so the variant must
reproduce the Euclidean variant's solution and residual estimates; and its bases must
satisfy their own defining relations."""
import numpy as np
import pytest

from oracle import sketch
from oracle.lowrank import rel_distance
from oracle.spksm import Space, spksm
from workloads import make_config


@pytest.mark.parametrize("k", [1, 2, 3])
def test_same_solution_as_euclidean_orthogonalisation(k):
    c = make_config("convdiff2d_1000", m=20, r=2)
    kw = dict(k=k, maxit=25, tol=0.0, p=5, s=800, seed=7, trunc_tol=0.0)
    a = spksm(c["A"], c["B"], c["C1"], c["C2"], **kw)
    b = spksm(c["A"], c["B"], c["C1"], c["C2"], orth="sketched", **kw)
    assert rel_distance(a.X1, a.X2, b.X1, b.X2) < 1e-10
    for (da, ra), (db, rb) in zip(a.history, b.history):
        assert da == db and abs(ra / rb - 1) < 1e-9


def test_basis_relations():
    """A U_d = U_{d+1} H_bar_d (truncated Arnoldi relation), and U_{d+1} is orthonormal in
    the sketched inner product and S-orthogonal to the window blocks."""
    c = make_config("reaction2d_500", m=16, r=2)
    n, r, k, d = c["n"], 2, 2, 10
    S = sketch.make("sparse_sign", n, 240, 8, 11)
    A = c["A"].to_scipy()
    sig = c["sigma"][:, None]
    sp_ = Space(lambda X: A @ X + sig * X, S, k, r, d, True, orth="sketched")
    sp_.init(c["C1"])
    for j in range(1, d + 1):
        sp_.step(j)
        SU = S @ sp_.blocks[j + 1]
        assert np.allclose(SU.T @ SU, np.eye(r), atol=1e-12)
        for i in range(max(1, j - k + 1), j + 1):
            assert np.abs((S @ sp_.blocks[i]).T @ SU).max() < 1e-12
    Ud = np.hstack([sp_.blocks[j] for j in range(1, d + 1)])
    Ud1 = np.hstack([sp_.blocks[j] for j in range(1, d + 2)])
    lhs = A @ Ud + sig * Ud
    assert np.linalg.norm(lhs - Ud1 @ sp_.H[:(d + 1) * r, :d * r]) < 1e-12 * np.linalg.norm(lhs)
