"""GPU parity on the paper's own workloads (Sec. 6) and on the general block step with a
long truncation window, through the C ABI.

* Example 6.1 (centered 2D convection-diffusion, w_A = (1, 1), w_B = (3y(1-x^2),
  -2x(1-y^2))) runs with k = 10 as in the paper's Table 2: k > 3 takes the general block
  step (block modified Gram-Schmidt over the window, fused SpMM / axpy / Gram kernels), for
  r = 1 and r = 3, both precisions, at a reduced grid.
* Example 6.3 (centered 3D convection-diffusion, Table 5) with k = 3, r = 1.
* Full orthogonalisation (t-PKSM with k >= d, Algorithm 2) against the oracle's full
  block Arnoldi Galerkin solution, which orthogonalises against all blocks twice and
  projects explicitly: with k >= d Algorithm 2 is full Arnoldi, so both must agree.

Bars as in the other parity tests: relative product distance <= 1e-6 (FP64 bulk) and
<= 1e-4 (mixed); residual estimates within 1e-6 / 1e-3 relative.
"""
import numpy as np
import pytest

from gpu_helpers import gpu_solve, history_ratio, oracle_solve, product_distance
from oracle.full_arnoldi import full_arnoldi_galerkin
from oracle.lowrank import rel_distance
from workloads import make_config

pytestmark = pytest.mark.gpu

TOL = {"fp64": (1e-6, 1e-6), "mixed": (1e-4, 1e-3)}


@pytest.mark.parametrize("r", [1, 3])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_ex61_k10_general_block_step(r, precision):
    cfg = make_config("ex61_convdiff2d_300", m=41, r=r)  # n = 1681, a ragged last tile
    prm = dict(k=10, maxit=30, p=10, s=8 * 31 * r, seed=cfg["sketch_seed"])
    print(f"ex61 m=41 r={r} k=10 {precision}", flush=True)
    g, _ = gpu_solve(cfg, precision=precision, tol=0.0, **prm)
    o = oracle_solve(cfg, tol=0.0, **prm)
    assert g.iters == o.d == prm["maxit"]
    tol_x, tol_h = TOL[precision]
    assert product_distance(g, o) <= tol_x
    assert history_ratio(g, o) <= tol_h


def test_ex61_k10_converged_run():
    """nu = 0.1, r = 1, k = 10 at n = 900 run to 1e-6: same stopping step as the oracle."""
    cfg = make_config("ex61_convdiff2d_300", m=30)
    prm = dict(k=10, maxit=200, p=10, s=1600, tol=1e-6, seed=cfg["sketch_seed"])
    print("ex61 m=30 converged", flush=True)
    g, _ = gpu_solve(cfg, **prm)
    o = oracle_solve(cfg, **prm)
    assert g.status == o.status == "converged"
    assert g.iters == o.d
    assert product_distance(g, o) <= 1e-6


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_ex63_fixed_d(precision):
    cfg = make_config("ex63_convdiff3d_100", m=13)  # n = 2197
    prm = dict(k=3, maxit=40, p=20, s=504, seed=cfg["sketch_seed"])
    print(f"ex63 m=13 {precision}", flush=True)
    g, _ = gpu_solve(cfg, precision=precision, tol=0.0, **prm)
    o = oracle_solve(cfg, tol=0.0, **prm)
    assert g.iters == o.d == prm["maxit"]
    tol_x, tol_h = TOL[precision]
    assert product_distance(g, o) <= tol_x
    assert history_ratio(g, o) <= tol_h


@pytest.mark.parametrize("name,m,r", [("convdiff2d_1000", 23, 2), ("ex61_convdiff2d_300", 25, 1)])
def test_full_orthogonalisation_equals_full_arnoldi(name, m, r):
    """t-PKSM with k = d = maxit orthogonalises every block against all earlier ones."""
    cfg = make_config(name, m=m, r=r)
    d = 16
    print(f"full Arnoldi {name} m={m} r={r} d={d}", flush=True)
    g, _ = gpu_solve(cfg, sketch="none", k=d, maxit=d, p=d, tol=0.0)
    X1, X2 = full_arnoldi_galerkin(cfg["A"], cfg["B"], cfg["C1"], cfg["C2"], d, sigma=cfg.get("sigma"))
    assert g.iters == d
    dist = rel_distance(g.X1.cpu().numpy(), g.X2.cpu().numpy(), X1, X2)
    assert dist <= 1e-6, dist


# The paper's stopping steps with p = 20 (Sec. 6, Table 2 for Ex. 6.1 at n = 90 000, Table 5
# for Ex. 6.3): soft pins.  The embedding (the subsampled randomized DCT, s = 1600 and 500)
# is the paper's kind but not its random draws, so the steps agree to within a few checks.
@pytest.mark.parametrize("nu,r,d_paper", [(0.1, 1, 480), (0.01, 3, 500), (0.001, 3, 760)])
def test_ex61_table2_stopping_steps(nu, r, d_paper):
    import paper_2311_16019_amd as skr
    from gpu_helpers import to_dev
    cfg = make_config("ex61_convdiff2d_300", nu=nu, r=r)
    prm = dict(k=10, maxit=1000, p=20, s=max(1600, 1001 * r), tol=1e-6, seed=cfg["sketch_seed"], sketch="srht")
    print(f"ex61 table 2: nu={nu} r={r}", flush=True)
    g, (A, B) = gpu_solve(cfg, **prm)
    print(f"  d={g.iters} (paper {d_paper}) rank={g.ell} failed checks={g.failed_checks}", flush=True)
    assert g.status == "converged"
    assert abs(g.iters - d_paper) <= 0.15 * d_paper
    tr = skr.true_residual(A, B, g.X1, g.X2, to_dev(cfg["C1"]), to_dev(cfg["C2"]))
    assert tr <= 5 * prm["tol"], tr


@pytest.mark.parametrize("m,d_paper", [(50, 140), (100, 220)])
def test_ex63_table5_stopping_steps(m, d_paper):
    import paper_2311_16019_amd as skr
    from gpu_helpers import to_dev
    cfg = make_config("ex63_convdiff3d_100", m=m)
    prm = dict(k=3, maxit=300, p=20, s=500, tol=1e-6, seed=cfg["sketch_seed"], sketch="srht")
    print(f"ex63 table 5: n={m ** 3}", flush=True)
    g, (A, B) = gpu_solve(cfg, **prm)
    print(f"  d={g.iters} (paper {d_paper}) rank={g.ell}", flush=True)
    assert g.status == "converged"
    assert abs(g.iters - d_paper) <= 0.3 * d_paper
    tr = skr.true_residual(A, B, g.X1, g.X2, to_dev(cfg["C1"]), to_dev(cfg["C2"]))
    assert tr <= 5 * prm["tol"], tr


def test_ex61_dependent_basis_falls_back_to_last_solved_check():
    """nu = 0.001, r = 1: the V space's truncated basis becomes numerically dependent near
    d = 320 (the condition number of its sketched triangular factor T passes 1e14 there in the
    oracle), and the sketched projected matrices of later checks have eigenvalue pairs the
    sign iteration cannot separate.  Those checks are skipped; at maxit the solve returns the
    factors of the last check that was solved, with status 'maxit', and those factors are
    consistent: their true residual is that check's estimate up to the embedding distortion."""
    import paper_2311_16019_amd as skr
    from gpu_helpers import to_dev
    cfg = make_config("ex61_convdiff2d_300", nu=0.001, r=1)
    prm = dict(k=10, maxit=400, p=20, s=1600, tol=1e-6, seed=cfg["sketch_seed"], sketch="srht")
    g, (A, B) = gpu_solve(cfg, **prm)
    print(f"  d={g.iters} status={g.status} failed checks={g.failed_checks} rho={g.rho_rel:.3e}", flush=True)
    assert g.status in ("maxit", "converged")
    if g.failed_checks:
        assert g.status == "maxit" and g.iters < prm["maxit"] and g.iters == g.history[-1][0]
    tr = skr.true_residual(A, B, g.X1, g.X2, to_dev(cfg["C1"]), to_dev(cfg["C2"]))
    assert 0.2 * g.rho_rel <= tr <= 5 * g.rho_rel, (tr, g.rho_rel)
