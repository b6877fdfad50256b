"""GPU parity of the sketched-inner-product orthogonalisation (orth = 'sketched': truncated
block Gram-Schmidt and QR in <x, y>_S = (S x)^T (S y), appendix A) against the FP64 oracle,
through the C ABI.

Same protocol and bars as the s-PKSM parity tests: fixed d on both sides, product distance
<= 1e-6 (FP64) / 1e-4 (mixed), residual estimates within 1e-6 / 1e-3 relative.  Because the
sketched Galerkin solution does not depend on the basis of the truncated space, the result
must also agree with the Euclidean variant to the same bars.
"""
import numpy as np
import pytest

from gpu_helpers import gpu_ops, gpu_solve, history_ratio, oracle_solve, product_distance, to_dev, torch_cuda
from oracle.lowrank import rel_distance
from oracle.lyapunov import spksm_lyapunov
from workloads import make_config

pytestmark = pytest.mark.gpu

TOL = {"fp64": (1e-6, 1e-6), "mixed": (1e-4, 1e-3)}

CASES = [
    ("laplace2d_64", 45, 1, dict(k=2, maxit=40, p=10, s=336, seed=3001)),
    ("convdiff2d_1000", 37, 4, dict(k=3, maxit=24, p=8, s=800, seed=3002)),
    ("reaction2d_500", 33, 2, dict(k=2, maxit=30, p=10, s=496, seed=3004)),
    ("aniso3d_100", 11, 3, dict(k=1, maxit=10, p=5, s=336, seed=3003)),
]


def _ids(c):
    return f"{c[0]}-m{c[1]}-r{c[2]}-k{c[3]['k']}"


@pytest.mark.parametrize("case", CASES, ids=_ids)
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_sketched_orth_fixed_d_parity(case, precision):
    name, m, r, prm = case
    cfg = make_config(name, m=m, r=r)
    print(f"sketched-orth case {name} m={m} r={r} {precision}", flush=True)
    g, _ = gpu_solve(cfg, precision=precision, tol=0.0, orth="sketched", **prm)
    o = oracle_solve(cfg, tol=0.0, orth="sketched", **prm)
    assert g.iters == o.d == prm["maxit"]
    tol_x, tol_h = TOL[precision]
    dist, hr = product_distance(g, o), history_ratio(g, o)
    assert dist <= tol_x, dist
    assert hr <= tol_h, hr
    # basis independence: the Euclidean variant of the oracle gives the same factors
    oe = oracle_solve(cfg, tol=0.0, **prm)
    assert product_distance(g, oe) <= tol_x


@pytest.mark.parametrize("recover", ["stored", "two_pass"])
def test_sketched_orth_converged_run(recover):
    cfg = make_config("convdiff2d_1000", m=40, r=2)
    prm = dict(k=2, maxit=150, p=5, tol=1e-7, s=1200, seed=3010)
    print(f"sketched-orth converged convdiff m=40 {recover}", flush=True)
    g, _ = gpu_solve(cfg, recover=recover, orth="sketched", **prm)
    o = oracle_solve(cfg, orth="sketched", **prm)
    assert g.status == o.status == "converged"
    assert g.iters == o.d
    assert product_distance(g, o) <= 1e-6
    assert history_ratio(g, o) <= 1e-6


def test_sketched_orth_lyapunov():
    import paper_2311_16019_amd as skr
    cfg = make_config("convdiff2d_1000", m=37, r=4)
    prm = dict(k=3, maxit=24, p=8, s=800, seed=3020, tol=0.0)
    for precision in ("fp64", "mixed"):
        print(f"sketched-orth Lyapunov convdiff m=37 {precision}", flush=True)
        A, _ = gpu_ops(cfg)
        g = skr.lyap_solve(A, to_dev(cfg["C1"]), precision=precision, orth="sketched", **prm)
        torch_cuda().cuda.synchronize()
        o = spksm_lyapunov(cfg["A"], cfg["C1"], sigma=cfg.get("sigma"), orth="sketched", **prm)
        assert g.iters == o.d == prm["maxit"]
        dist = rel_distance(g.X1.cpu().numpy(), g.X2.cpu().numpy(), o.X1, o.X2)
        assert dist <= TOL[precision][0], (precision, dist)
        assert history_ratio(g, o) <= TOL[precision][1]


def test_sketched_orth_breakdown_on_invariant_krylov_space():
    """A has three distinct eigenvalues, so K_3(A, C1) is invariant.  A is symmetric but not
    in the sketched inner product, so only a window that spans all three blocks (k = 3)
    leaves a zero remainder at d = 3; with k = 2 neither side breaks down."""
    import scipy.sparse as sp
    from workloads.stencil import CSR
    n = 300
    A = CSR.from_scipy(sp.diags(np.tile([1.0, 2.0, 4.0], n // 3)))
    rng = np.random.Generator(np.random.PCG64(1))
    B = CSR.from_scipy(sp.diags(np.linspace(1, 3, n)) + sp.random(n, n, density=0.01, random_state=3))
    cfg = dict(A=A, B=B, sigma=None, C1=rng.standard_normal((n, 1)), C2=rng.standard_normal((n, 1)))
    prm = dict(k=3, maxit=10, p=5, s=96, tol=0.0, seed=5)
    print("sketched-orth breakdown n=300", flush=True)
    g, _ = gpu_solve(cfg, orth="sketched", **prm)
    o = oracle_solve(cfg, orth="sketched", **prm)
    assert g.status == o.status == "breakdown"
    assert g.iters == o.d == 3
    assert product_distance(g, o) <= 1e-6


def test_sketched_orth_unsupported_requests():
    import paper_2311_16019_amd as skr
    cfg = make_config("convdiff2d_1000", m=10, r=2)
    A, B = gpu_ops(cfg)
    C1, C2 = to_dev(cfg["C1"]), to_dev(cfg["C2"])
    with pytest.raises(skr.SkrError) as ei:  # no embedding: no sketched inner product
        skr.solve(A, B, C1, C2, maxit=5, p=5, sketch="none", orth="sketched")
    assert ei.value.code == -1
    with pytest.raises(skr.SkrError) as ei:  # window beyond the two-pass step's
        skr.solve(A, B, C1, C2, maxit=5, p=5, s=48, k=4, orth="sketched")
    assert ei.value.code == -4


def test_sketched_orth_full_size_convdiff_fixed_d():
    """The 1000 x 1000 convection-diffusion pair (n = 1e6, r = 4, k = 3, s = 8000) at the
    benchmark's launch configuration, compared with the oracle at d = 20."""
    cfg = make_config("convdiff2d_1000")
    prm = dict(k=3, maxit=20, p=20, s=cfg["s"], tol=0.0, seed=cfg["sketch_seed"])
    o = None
    for precision in ("fp64", "mixed"):
        print(f"sketched-orth full-size convdiff {precision}", flush=True)
        g, _ = gpu_solve(cfg, precision=precision, orth="sketched", **prm)
        if o is None:
            o = oracle_solve(cfg, orth="sketched", **prm)
        dist = product_distance(g, o)
        assert dist <= TOL[precision][0], (precision, dist)
        assert history_ratio(g, o) <= TOL[precision][1]
