"""GPU: the library's device-memory cache and stream reuse across calls.

Consecutive solves take their workspaces from blocks that earlier solves released (and
from streams they used); results must not depend on that.  Runs of one problem are compared
with each other and against the oracle, with a solve of another size and a cache release in
between; every reduction adds in a fixed order, so repeated solves agree bit for bit.
"""
import pytest

from gpu_helpers import gpu_solve, oracle_solve, product_distance
from oracle.lowrank import rel_distance
from workloads import make_config

pytestmark = pytest.mark.gpu


def _dist(a, b):
    return rel_distance(a.X1.cpu().numpy(), a.X2.cpu().numpy(), b.X1.cpu().numpy(), b.X2.cpu().numpy())


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_reused_workspaces_give_the_same_solution(precision):
    import paper_2311_16019_amd as skr

    cfg = make_config("convdiff2d_1000", m=37, r=4)
    small = make_config("laplace2d_64", m=21, r=2)
    prm = dict(k=3, maxit=24, p=8, s=800, seed=1002, tol=0.0, precision=precision)
    print(f"runtime reuse {precision}", flush=True)
    first, _ = gpu_solve(cfg, **prm)
    gpu_solve(small, k=2, maxit=12, p=6, s=96, seed=7, tol=0.0, precision=precision)
    second, _ = gpu_solve(cfg, **prm)
    skr.release_cached_memory()
    third, _ = gpu_solve(cfg, **prm)
    bar = 1e-9 if precision == "fp64" else 1e-5
    assert _dist(first, second) <= bar
    assert _dist(first, third) <= bar
    o = oracle_solve(cfg, **prm)
    assert product_distance(second, o) <= (1e-6 if precision == "fp64" else 1e-4)


@pytest.mark.parametrize("precision,k", [("fp64", 3), ("mixed", 3), ("fp64", 10), ("mixed", 10)])
def test_repeated_solves_are_bitwise_identical(precision, k):
    """Every reduction of a solve (block products, sketch, sketched QR update, projected
    solve, recovery) adds in a fixed order: two solves of the same problem give the same
    factors and residual history bit for bit (needed by the fixed-d finite-difference check
    of the gradients)."""
    import paper_2311_16019_amd as skr
    from gpu_helpers import gpu_ops, to_dev, torch_cuda
    from workloads import make_config
    torch = torch_cuda()
    cfg = make_config("convdiff2d_1000", m=61, r=4)
    A, B = gpu_ops(cfg)
    C1, C2 = to_dev(cfg["C1"]), to_dev(cfg["C2"])
    prm = dict(k=k, maxit=60, p=20, s=968, tol=0.0, seed=cfg["sketch_seed"], precision=precision)
    a = skr.solve(A, B, C1, C2, **prm)
    b = skr.solve(A, B, C1, C2, **prm)
    assert a.history == b.history
    assert torch.equal(a.X1, b.X1) and torch.equal(a.X2, b.X2)
