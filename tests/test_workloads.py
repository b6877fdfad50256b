"""Pins of the workload operators of the paper's Examples 6.1 and 6.3 (Sec. 6): the
centered finite differences are consistent (second order) with the continuous
convection-diffusion operator, so a wrong sign, index or scale of a diffusion or
convection entry fails."""
import numpy as np
import pytest

from workloads import convdiff_centered, make_config
from workloads.configs import ex61_velocities, ex63_velocities


def _apply_error(m, dim, nu, wfun, u, lu):
    """max |A u_h - L(u)| at the nodes, relative to max |L(u)|."""
    A = convdiff_centered(m, dim, nu, wfun).to_scipy()
    h = 1.0 / (m + 1)
    x = (np.arange(m) + 1) * h
    grids = np.meshgrid(*([x] * dim), indexing="ij")[::-1]
    uh = u(*grids).ravel()
    ref = lu(*grids).ravel()
    return np.max(np.abs(A @ uh - ref)) / np.max(np.abs(ref))


def test_centered_2d_is_second_order_with_example_61_velocities():
    nu = 0.1
    wa, wb = ex61_velocities()
    pi = np.pi
    u = lambda x, y: np.sin(pi * x) * np.sin(2 * pi * y)
    ux = lambda x, y: pi * np.cos(pi * x) * np.sin(2 * pi * y)
    uy = lambda x, y: 2 * pi * np.sin(pi * x) * np.cos(2 * pi * y)
    lap = lambda x, y: -5 * pi**2 * u(x, y)
    for w in (wa, wb):
        def lu(x, y, w=w):
            wx, wy = w(x, y)
            return -nu * lap(x, y) + wx * ux(x, y) + wy * uy(x, y)
        e1 = _apply_error(40, 2, nu, w, u, lu)
        e2 = _apply_error(80, 2, nu, w, u, lu)
        assert e1 < 5e-3
        assert 3.5 < e1 / e2 < 4.5  # h^2 convergence


def test_centered_3d_is_second_order_with_example_63_velocities():
    nu = 0.005
    wa, wb = ex63_velocities()
    pi = np.pi
    u = lambda x, y, z: np.sin(pi * x) * np.sin(pi * y) * np.sin(pi * z)
    grad = lambda x, y, z: (pi * np.cos(pi * x) * np.sin(pi * y) * np.sin(pi * z),
                            pi * np.sin(pi * x) * np.cos(pi * y) * np.sin(pi * z),
                            pi * np.sin(pi * x) * np.sin(pi * y) * np.cos(pi * z))
    for w in (wa, wb):
        def lu(x, y, z, w=w):
            g = grad(x, y, z)
            wc = w(x, y, z)
            return nu * 3 * pi**2 * u(x, y, z) + sum(wc[c] * g[c] for c in range(3))
        e1 = _apply_error(16, 3, nu, w, u, lu)
        e2 = _apply_error(32, 3, nu, w, u, lu)
        assert e1 < 2e-2
        assert 3.2 < e1 / e2 < 4.8


def test_centered_operator_structure():
    # constant velocity: A - A^T is the convection part, antisymmetric with entries w/h
    m, nu = 6, 0.3
    A = convdiff_centered(m, 2, nu, lambda x, y: (np.full_like(x, 2.0), np.full_like(x, -1.0))).to_scipy()
    h = 1.0 / (m + 1)
    S = (A + A.T) / 2
    K = (A - A.T) / 2
    assert np.allclose(S.diagonal(), 4 * nu / h**2)
    assert np.isclose(K[0, 1], 2.0 / (2 * h)) and np.isclose(K[0, m], -1.0 / (2 * h))
    assert A.nnz == 5 * m * m - 4 * m


@pytest.mark.parametrize("name,n,nnz", [("ex61_convdiff2d_300", 90000, 5 * 300**2 - 4 * 300),
                                        ("ex63_convdiff3d_100", 10**6, 7 * 100**3 - 6 * 100**2)])
def test_paper_workload_sizes(name, n, nnz):
    cfg = make_config(name, m=8)
    assert cfg["n"] == 8 ** (2 if "2d" in name else 3)
    full = dict(ex61_convdiff2d_300=300, ex63_convdiff3d_100=100)[name]
    dim = 2 if "2d" in name else 3
    assert full**dim == n
    assert nnz == (5 * full**2 - 4 * full if dim == 2 else 7 * full**3 - 6 * full**2)
    C1, C2 = cfg["C1"], cfg["C2"]
    assert np.isclose(np.linalg.norm(C1 @ C2.T), 1.0)
