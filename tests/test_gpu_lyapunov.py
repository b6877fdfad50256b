"""GPU parity of the Lyapunov specialisation (skr_lyap_solve: one Krylov space, B = A^T,
C2 = C1) against the FP64 oracle, through the C ABI; same bars as the Sylvester tests."""
import numpy as np
import pytest
import scipy.sparse as sp

from gpu_helpers import gpu_ops, history_ratio, to_dev, torch_cuda
from oracle.lowrank import rel_distance, true_residual
from oracle.lyapunov import spksm_lyapunov, tpksm_lyapunov
from workloads import make_config

pytestmark = pytest.mark.gpu

TOL = {"fp64": (1e-6, 1e-6), "mixed": (1e-4, 1e-3)}

CASES = [
    ("laplace2d_64", 45, 1, dict(k=2, maxit=40, p=10, s=336, seed=2001)),
    ("convdiff2d_1000", 37, 4, dict(k=3, maxit=24, p=8, s=800, seed=2002)),
    ("reaction2d_500", 33, 2, dict(k=2, maxit=30, p=10, s=496, seed=2004)),
]


def _gpu(cfg, **prm):
    import paper_2311_16019_amd as skr
    A, _ = gpu_ops(cfg)
    res = skr.lyap_solve(A, to_dev(cfg["C1"]), **prm)
    torch_cuda().cuda.synchronize()
    return res


def _oracle(cfg, sketch="sparse_sign", **prm):
    prm = dict(prm)
    prm.pop("precision", None)
    if sketch == "none":
        for key in ("s", "seed"):
            prm.pop(key, None)
        return tpksm_lyapunov(cfg["A"], cfg["C1"], sigma=cfg.get("sigma"), **prm)
    return spksm_lyapunov(cfg["A"], cfg["C1"], sigma=cfg.get("sigma"), **prm)


def _dist(g, o):
    return rel_distance(g.X1.cpu().numpy(), g.X2.cpu().numpy(), o.X1, o.X2)


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[0]}-m{c[1]}-r{c[2]}")
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("sketch", ["sparse_sign", "none"])
def test_lyapunov_fixed_d_parity(case, precision, sketch):
    name, m, r, prm = case
    cfg = make_config(name, m=m, r=r)
    print(f"Lyapunov case {name} m={m} r={r} {precision} {sketch}", flush=True)
    g = _gpu(cfg, precision=precision, tol=0.0, sketch=sketch, **prm)
    o = _oracle(cfg, sketch=sketch, tol=0.0, **prm)
    assert g.iters == o.d == prm["maxit"]
    tol_x, tol_h = TOL[precision]
    assert _dist(g, o) <= tol_x
    assert history_ratio(g, o) <= tol_h
    X = g.X1.cpu().numpy() @ g.X2.cpu().numpy().T
    assert np.linalg.norm(X - X.T) <= 1e-10 * np.linalg.norm(X)  # the solution is symmetric


def test_lyapunov_converged_run():
    cfg = make_config("reaction2d_500", m=30, r=2)
    prm = dict(k=2, maxit=300, p=5, s=2408, seed=2011, tol=1e-8)
    print("Lyapunov converged reaction m=30", flush=True)
    g = _gpu(cfg, **prm)
    o = _oracle(cfg, **prm)
    assert g.status == o.status == "converged"
    assert g.iters == o.d
    assert _dist(g, o) <= 1e-6
    As = cfg["A"].to_scipy() + sp.diags(cfg["sigma"])
    tr = true_residual(As, As.T.tocsr(), cfg["C1"], cfg["C1"], g.X1.cpu().numpy(), g.X2.cpu().numpy())
    assert tr <= 1e-7
