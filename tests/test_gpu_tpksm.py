"""GPU parity of t-PKSM (Algorithm 2: the truncated Arnoldi method, no embedding) against
the FP64 oracle, through the C ABI (sketch = SKR_SKETCH_NONE).

Same protocol and bars as the s-PKSM parity tests: fixed d on both sides, product distance
<= 1e-6 (FP64) / 1e-4 (mixed), residual estimates within 1e-6 / 1e-3 relative.
"""
import pytest

from gpu_helpers import gpu_solve, history_ratio, product_distance
from oracle.lowrank import true_residual
from oracle.tpksm import tpksm
from workloads import make_config

pytestmark = pytest.mark.gpu

TOL = {"fp64": (1e-6, 1e-6), "mixed": (1e-4, 1e-3)}

CASES = [
    ("laplace2d_64", 45, 1, dict(k=2, maxit=40, p=10)),
    ("convdiff2d_1000", 37, 4, dict(k=3, maxit=24, p=8)),
    ("aniso3d_100", 11, 8, dict(k=2, maxit=10, p=5)),
    ("reaction2d_500", 33, 2, dict(k=2, maxit=30, p=10)),
]


def _oracle(cfg, **prm):
    prm = dict(prm)
    prm.pop("precision", None)
    prm.pop("sketch", None)
    return tpksm(cfg["A"], cfg["B"], cfg["C1"], cfg["C2"], sigma=cfg.get("sigma"), **prm)


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[0]}-m{c[1]}-r{c[2]}")
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_tpksm_fixed_d_parity(case, precision):
    name, m, r, prm = case
    cfg = make_config(name, m=m, r=r)
    print(f"t-PKSM case {name} m={m} r={r} {precision}", flush=True)
    g, _ = gpu_solve(cfg, precision=precision, tol=0.0, sketch="none", **prm)
    o = _oracle(cfg, tol=0.0, **prm)
    assert g.iters == o.d == prm["maxit"]
    tol_x, tol_h = TOL[precision]
    assert product_distance(g, o) <= tol_x
    assert history_ratio(g, o) <= tol_h


@pytest.mark.parametrize("recover", ["stored", "two_pass"])
def test_tpksm_converged_run(recover):
    cfg = make_config("laplace2d_64", m=30)
    prm = dict(k=3, maxit=300, p=5, tol=1e-7)
    print(f"t-PKSM converged laplace m=30 {recover}", flush=True)
    g, _ = gpu_solve(cfg, sketch="none", recover=recover, **prm)
    o = _oracle(cfg, **prm)
    assert g.status == o.status == "converged"
    assert g.iters == o.d
    assert product_distance(g, o) <= 1e-6
    tr = true_residual(cfg["A"], cfg["B"], cfg["C1"], cfg["C2"], g.X1.cpu().numpy(), g.X2.cpu().numpy())
    assert tr <= 1e-7 * (1 + 1e-6)
