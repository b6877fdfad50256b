"""Pins for the oracle's gradients of L = tr(P1^T X P2) through the Sylvester solve."""
import numpy as np

from oracle.adjoint import dense_grads, solve_and_grad
from oracle.spksm import spksm
from oracle.sylvester import bartels_stewart
from workloads import make_config


def _case(m=6):
    c = make_config("reaction2d_500", m=m, r=2)
    rng = np.random.Generator(np.random.PCG64(99))
    P1 = rng.standard_normal((c["n"], 3))
    P2 = rng.standard_normal((c["n"], 3))
    return c, P1, P2


def _dense_loss(c, C1, C2, sigma, P1, P2):
    A = c["A"].to_scipy().toarray() + np.diag(sigma)
    X = bartels_stewart(A, c["B"].to_scipy().toarray(), C1 @ C2.T)
    return float(np.sum(P1 * (X @ P2)))


def test_dense_gradients_match_central_differences():
    """The adjoint formulas (dC1 = Lam C2, dC2 = Lam^T C1, dsigma = -rowsum(Lam o X)) against
    central finite differences of the dense solve along random directions."""
    c, P1, P2 = _case()
    g = dense_grads(c["A"], c["B"], c["C1"], c["C2"], c["sigma"], P1, P2)
    rng = np.random.Generator(np.random.PCG64(7))
    eps = 1e-6
    for which in ("C1", "C2", "sigma"):
        for _ in range(3):
            args = dict(C1=c["C1"].copy(), C2=c["C2"].copy(), sigma=c["sigma"].copy())
            delta = rng.standard_normal(args[which].shape)
            plus = {k: v + (eps * delta if k == which else 0) for k, v in args.items()}
            minus = {k: v - (eps * delta if k == which else 0) for k, v in args.items()}
            fd = (_dense_loss(c, plus["C1"], plus["C2"], plus["sigma"], P1, P2)
                  - _dense_loss(c, minus["C1"], minus["C2"], minus["sigma"], P1, P2)) / (2 * eps)
            an = float(np.sum(g["d" + which] * delta))
            assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-12), (which, fd, an)


def test_spksm_gradients_match_dense_adjoint():
    c, P1, P2 = _case(m=8)
    g = solve_and_grad(c["A"], c["B"], c["C1"], c["C2"], c["sigma"], P1, P2,
                       k=2, maxit=30, tol=1e-11, p=1, s=160, seed=4)
    ref = dense_grads(c["A"], c["B"], c["C1"], c["C2"], c["sigma"], P1, P2)
    for key in ("dC1", "dC2", "dsigma", "dP1", "dP2"):
        err = np.linalg.norm(g[key] - ref[key]) / np.linalg.norm(ref[key])
        assert err < 1e-7, (key, err)
    assert abs(g["loss"] - ref["loss"]) < 1e-8 * abs(ref["loss"])


def test_adjoint_of_symmetric_problem_reproduces_forward():
    """A and B symmetric: with P1 = C1, P2 = C2 the adjoint run is the forward run."""
    c = make_config("laplace2d_64", m=10)
    kw = dict(k=2, maxit=20, tol=1e-10, p=2, s=80, seed=3)
    f = spksm(c["A"], c["B"], c["C1"], c["C2"], **kw)
    A_t = c["A"].transpose()
    B_t = c["B"].transpose()
    a = spksm(A_t, B_t, c["C1"], c["C2"], **kw)
    assert f.d == a.d
    assert np.allclose(f.X1 @ f.X2.T, a.X1 @ a.X2.T, rtol=0, atol=1e-14 * np.abs(f.X1 @ f.X2.T).max())


def test_fixed_d_spksm_finite_differences():
    """Central differences of the s-PKSM loss at a fixed iteration count d (same S) agree
    with its adjoint gradient once both solves are converged well below the FD error."""
    c, P1, P2 = _case(m=8)
    kw = dict(k=2, maxit=30, tol=1e-12, p=1, s=160, seed=4)
    g = solve_and_grad(c["A"], c["B"], c["C1"], c["C2"], c["sigma"], P1, P2, **kw)
    d = g["fwd"].d
    fixed = dict(kw, maxit=d, tol=0.0)
    rng = np.random.Generator(np.random.PCG64(8))
    eps = 1e-6
    for _ in range(3):
        delta = rng.standard_normal(c["n"])
        lp = spksm(c["A"], c["B"], c["C1"], c["C2"], sigma=c["sigma"] + eps * delta, **fixed)
        lm = spksm(c["A"], c["B"], c["C1"], c["C2"], sigma=c["sigma"] - eps * delta, **fixed)
        Lp = float(np.sum((P1.T @ lp.X1) * (P2.T @ lp.X2)))
        Lm = float(np.sum((P1.T @ lm.X1) * (P2.T @ lm.X2)))
        fd = (Lp - Lm) / (2 * eps)
        an = float(np.sum(g["dsigma"] * delta))
        assert abs(fd - an) <= 1e-5 * abs(an)
