"""Parity at the full sizes of the two other benchmark-scale workloads, through the C ABI:
the 3D anisotropic pair (n = 1e6, r = 8, k = 2, s = 9600) and the log-normal diffusion
operator (n = 4e6, r = 10, k = 2, s = 4000).  Both have r > 4, so they run the general block
step (block MGS with the fused SpMM / axpy / Gram kernels) at the size where its launch
configuration is the one a production run uses.  The oracle runs a few block steps at the
same size; bars as in the other parity tests."""
import pytest

from gpu_helpers import gpu_solve, history_ratio, oracle_solve, product_distance
from workloads import make_config

pytestmark = pytest.mark.gpu

TOL = {"fp64": (1e-6, 1e-6), "mixed": (1e-4, 1e-3)}


def test_full_size_aniso3d_fixed_d():
    cfg = make_config("aniso3d_100")
    prm = dict(k=cfg["k"], maxit=6, p=6, s=cfg["s"], tol=0.0, seed=cfg["sketch_seed"])
    o = oracle_solve(cfg, **prm)
    for precision in ("fp64", "mixed"):
        print(f"full-size aniso3d {precision}", flush=True)
        g, _ = gpu_solve(cfg, precision=precision, **prm)
        assert g.iters == o.d == prm["maxit"]
        assert product_distance(g, o) <= TOL[precision][0]
        assert history_ratio(g, o) <= TOL[precision][1]


def test_full_size_lognormal_fixed_d():
    cfg = make_config("lognormal2d_2000")
    prm = dict(k=cfg["k"], maxit=4, p=4, s=cfg["s"], tol=0.0, seed=cfg["sketch_seed"])
    print("full-size lognormal mixed", flush=True)
    g, _ = gpu_solve(cfg, precision="mixed", **prm)
    o = oracle_solve(cfg, **prm)
    assert g.iters == o.d == prm["maxit"]
    assert product_distance(g, o) <= TOL["mixed"][0]
    assert history_ratio(g, o) <= TOL["mixed"][1]
