"""The gradient check of the differentiation workload at full size, on the GPU: the
500 x 500 Laplacian plus diag(sigma) against the Laplacian (n = 250 000, r = 2), loss
L = tr(P1^T X P2) with P1, P2 n x 4 Gaussian.

Protocol: the forward and the adjoint solves run to a relative residual estimate of 1e-11
(the gradients inherit the solves' error times the equation's conditioning: at 1e-8 the
difference quotients disagreed by 3e-5);
the adjoint factors give dL/dC1, dL/dC2 and dL/dsigma.  Central finite differences of L
use forward solves with the base solve's stopping step d* held fixed (tol = 0, maxit = d*)
and the same embeddings, so that L is a smooth function of the data (a changed stopping
step or embedding would make the difference quotient measure noise); every reduction of a
solve adds in a fixed order, so the two solves of a difference differ only through the data.

Directions: three Gaussian ones each in C1 and C2 (step 1e-4 of the factor's size: each
solve's L carries rounding noise of about 1e-11 of L, which steps of 1e-6 turned into
quotient errors of 1e-5, and L depends on C only weakly nonlinearly through the Krylov
space, so the central difference's own error stays far below that); for
sigma, directions the solution responds to: the constant shift, sigma itself, the smooth
bump sin(pi x) sin(pi y), and two Gaussian bumps (width 25 grid points) around the
grid points with the largest |dL/dsigma|.  A Gaussian direction in sigma or a single
coordinate moves L by only about 3e-11 and 5e-13 per unit step (the smooth low modes that
carry X average such a direction out), and their difference quotients were measured to be
noise (relative errors of 4e-2 to 5); the smooth directions move L by about 1e-9 per unit.
The error of a Gaussian direction is taken relative to ||grad||_F, the root mean square of
<grad, delta> over such directions (a direction nearly orthogonal to the gradient would
otherwise turn the same absolute error into a large relative one); that of a sigma direction
relative to <grad, delta>.
"""
import numpy as np
import pytest

from gpu_helpers import to_dev, torch_cuda
from workloads import make_config

pytestmark = pytest.mark.gpu


@pytest.mark.timeout(900)
def test_fixed_d_finite_differences_match_adjoint_gradients():
    import paper_2311_16019_amd as skr
    torch = torch_cuda()
    cfg = make_config("reaction2d_500")
    n, r = cfg["n"], cfg["r"]
    A = skr.Operator.from_csr(cfg["A"].indptr, cfg["A"].indices, cfg["A"].data, diag=cfg["sigma"])
    B = skr.Operator.from_csr(cfg["B"].indptr, cfg["B"].indices, cfg["B"].data)
    C1, C2, P1, P2 = (to_dev(cfg[k]) for k in ("C1", "C2", "P1", "P2"))
    sig = to_dev(cfg["sigma"])
    base = dict(k=cfg["k"], p=100, maxit=2500, s=cfg["s"], seed=cfg["sketch_seed"])
    f = skr.solve(A, B, C1, C2, tol=1e-11, **base)
    # the adjoint block has the 4 columns of P1, P2: twice the sketch rows
    a = skr.adjoint_solve(A, B, P1, P2, tol=1e-11, **dict(base, s=2 * cfg["s"]))
    assert f.status == a.status == "converged"
    d_star = f.iters
    g = skr.pairing_grads(f.X1, f.X2, C1, C2, P1, P2, L1=a.X1, L2=a.X2)
    fixed = dict(base, maxit=d_star, p=d_star, tol=0.0)
    print(f"d* = {d_star}, adjoint d = {a.iters}", flush=True)

    def loss(c1, c2, sg):
        A.set_diag(sg)
        x = skr.solve(A, B, c1, c2, **fixed)
        assert x.iters == d_star
        return skr.pairing_grads(x.X1, x.X2, c1, c2, P1, P2, want=())["loss"]

    rng = np.random.Generator(np.random.PCG64(2024))
    m = cfg["m"]
    x = np.arange(1, m + 1) / (m + 1)
    xx, yy = np.meshgrid(x, x, indexing="ij")  # row-major grid, index i * m + j

    def bump(idx, width=25.0):
        i0, j0 = divmod(idx, m)
        ii, jj = np.meshgrid(np.arange(m), np.arange(m), indexing="ij")
        return np.exp(-((ii - i0) ** 2 + (jj - j0) ** 2) / (2 * width ** 2)).ravel()

    top = torch.argsort(torch.abs(g["dsig"]), descending=True)[:2].tolist()
    sig_dirs = [("sigma_const", np.ones(n)), ("sigma_self", cfg["sigma"]),
                ("sigma_sine", (np.sin(np.pi * xx) * np.sin(np.pi * yy)).ravel())]
    sig_dirs += [(f"sigma_bump{i}", bump(i)) for i in top]
    cases = [(w, to_dev(rng.standard_normal((n, r)))) for w in ("C1",) * 3 + ("C2",) * 3]
    cases += [(w, to_dev(v)) for w, v in sig_dirs]
    errs = []
    for which, delta in cases:
        if which.startswith("sigma"):
            # steps of 1e-2 on sigma's scale of one against the low eigenvalues of the operator
            # pair (about 40): the central difference's error (eps / 40)^2 ~ 1e-7 and the
            # rounding noise both stay well below the bar (steps of 1e-3 left 1e-5 of noise)
            eps = 1e-2 / float(torch.max(torch.abs(delta)))
            grad = g["dsig"]
        else:
            x0, grad = (C1, g["dC1"]) if which == "C1" else (C2, g["dC2"])
            eps = 1e-4 * float(torch.linalg.norm(x0)) / float(torch.linalg.norm(delta))

        def moved(sgn):
            step = sgn * eps * delta
            return (C1 + step if which == "C1" else C1, C2 + step if which == "C2" else C2,
                    sig + step if which.startswith("sigma") else sig)

        fd = (loss(*moved(1.0)) - loss(*moved(-1.0))) / (2 * eps)
        an = float(torch.sum(grad * delta))
        scale = abs(an) if which.startswith("sigma") else float(torch.linalg.norm(grad))
        errs.append((which, abs(fd - an) / scale))
        print(f"  {which}: fd {fd:.10e} adjoint {an:.10e} rel {errs[-1][1]:.2e}", flush=True)
    A.set_diag(sig)
    assert max(e for _, e in errs) <= 1e-5, errs
