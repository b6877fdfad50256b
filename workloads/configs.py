"""The five benchmark workloads, with full sizes and a grid-size override for tests.

Every entry states the operator pair, the block size ``r``, the truncation ``k``,
``maxit``, the sketch size ``s``, the relative tolerance and the check period ``p``.
``make_config(name, m=...)`` rebuilds the same workload family on a smaller grid;
``s`` then follows the workload's formula in ``maxit * r``.
"""
from __future__ import annotations

import numpy as np

from .factors import gaussian_block, gaussian_factors
from .stencil import (
    convdiff_2d_upwind,
    convdiff_centered,
    diffusion_3d,
    laplacian_2d,
    lognormal_field_2d,
    vardiff_2d,
)

# name -> full-size description
CONFIGS = {
    # 2D Dirichlet Laplacian, A = B, closed-form solution available.
    "laplace2d_64": dict(dim=2, m=64, r=1, k=2, maxit=100, s_per=2, tol=1e-8, p=20,
                         rhs_seed=11, sketch_seed=1001),
    # 2D upwind convection-diffusion pair, FP64 and mixed precision.
    "convdiff2d_1000": dict(dim=2, m=1000, r=4, k=3, maxit=500, s_per=4, tol=1e-6, p=20,
                            rhs_seed=12, sketch_seed=1002, loss_seed=32),
    # 3D anisotropic diffusion vs isotropic Laplacian + I.
    "aniso3d_100": dict(dim=3, m=100, r=8, k=2, maxit=600, s_per=2, tol=1e-6, p=20,
                        rhs_seed=13, sketch_seed=1003),
    # 2D Laplacian + diag(sigma) vs Laplacian: differentiation workload.
    "reaction2d_500": dict(dim=2, m=500, r=2, k=2, maxit=2500, s_per=2, tol=1e-8, p=100,
                           rhs_seed=14, sketch_seed=1004, sigma_seed=24, loss_seed=34),
    # 2D log-normal variable-coefficient diffusion, A = B.
    "lognormal2d_2000": dict(dim=2, m=2000, r=10, k=2, maxit=200, s_per=2, tol=1e-6, p=20,
                             rhs_seed=15, sketch_seed=1005, field_seed=45, loss_seed=35),
    # The paper's Example 6.1 (Sec. 6, Table 2): centered 2D convection-diffusion on 300^2
    # nodes, w_A = (1, 1), w_B = (3y(1-x^2), -2x(1-y^2)), nu in {0.1, 0.01, 0.001},
    # r in {1, 3}, k = 10, s = 1600, maxit = 800, tol 1e-6, p in {1, 20}.
    "ex61_convdiff2d_300": dict(dim=2, m=300, r=1, k=10, maxit=800, s=1600, tol=1e-6, p=20, nu=0.1,
                                rhs_seed=16, sketch_seed=1006),
    # The paper's Example 6.3 (Sec. 6, Table 5): centered 3D convection-diffusion, nu = 0.005,
    # w_A = (x sin x, y cos y, exp(z^2 - 1)), w_B = ((1 - x^2) y z, 1, exp(z)), n = m^3 with
    # m in {50, 60, 70, 80, 90, 100}; r = 1, k = 3, s = 500, maxit = 250, tol 1e-6.
    "ex63_convdiff3d_100": dict(dim=3, m=100, r=1, k=3, maxit=250, s=500, tol=1e-6, p=20, nu=0.005,
                                rhs_seed=17, sketch_seed=1007),
}


def ex61_velocities():
    """Convection fields of Example 6.1 (Sec. 6): ``w_A = (1, 1)``, ``w_B = (3y(1-x^2), -2x(1-y^2))``."""
    wa = lambda x, y: (np.ones_like(x), np.ones_like(x))
    wb = lambda x, y: (3.0 * y * (1.0 - x * x), -2.0 * x * (1.0 - y * y))
    return wa, wb


def ex63_velocities():
    """Convection fields of Example 6.3 (Sec. 6): ``w_A = (x sin x, y cos y, e^{z^2-1})``,
    ``w_B = ((1-x^2) y z, 1, e^z)``."""
    wa = lambda x, y, z: (x * np.sin(x), y * np.cos(y), np.exp(z * z - 1.0))
    wb = lambda x, y, z: ((1.0 - x * x) * y * z, np.ones_like(x), np.exp(z))
    return wa, wb

NU_CONVDIFF = 1e-2
W_A = (1.0, 0.5)
W_B = (-0.3, 1.0)
ANISO = (1.0, 10.0, 100.0)
CORR_LEN = 0.1


def make_config(name: str, m: int | None = None, maxit: int | None = None, r: int | None = None,
                nu: float | None = None) -> dict:
    """Build a workload: operators ``A``, ``B`` (CSR), factors and solver parameters.

    ``A`` may come with a separate nonnegative diagonal ``sigma`` (the reaction
    workload): the equation is then ``(A0 + diag(sigma)) X + X B = C1 C2^T`` and the
    returned ``A`` is ``A0`` with ``sigma`` given separately.
    """
    c = dict(CONFIGS[name])
    if m is not None:
        c["m"] = m
    if maxit is not None:
        c["maxit"] = maxit
    if r is not None:
        c["r"] = r
    if nu is not None:
        c["nu"] = nu
    mm = c["m"]
    sigma = None
    if name.startswith("laplace2d"):
        A = laplacian_2d(mm)
        B = A
    elif name.startswith("convdiff2d"):
        A = convdiff_2d_upwind(mm, NU_CONVDIFF, W_A)
        B = convdiff_2d_upwind(mm, NU_CONVDIFF, W_B)
    elif name.startswith("aniso3d"):
        A = diffusion_3d(mm, ANISO)
        B = diffusion_3d(mm, (1.0, 1.0, 1.0), shift=1.0)
    elif name.startswith("reaction2d"):
        A = laplacian_2d(mm)
        B = A
        rng = np.random.Generator(np.random.PCG64(c["sigma_seed"]))
        sigma = rng.uniform(0.0, 1.0, size=A.n)
    elif name.startswith("ex61"):
        wa, wb = ex61_velocities()
        A = convdiff_centered(mm, 2, c["nu"], wa)
        B = convdiff_centered(mm, 2, c["nu"], wb)
    elif name.startswith("ex63"):
        wa, wb = ex63_velocities()
        A = convdiff_centered(mm, 3, c["nu"], wa)
        B = convdiff_centered(mm, 3, c["nu"], wb)
    elif name.startswith("lognormal2d"):
        kappa = lognormal_field_2d(mm, CORR_LEN, c["field_seed"])
        A = vardiff_2d(kappa)
        B = A
    else:
        raise KeyError(name)
    n = A.n
    C1, C2 = gaussian_factors(n, B.n, c["r"], c["rhs_seed"])
    out = dict(name=name, A=A, B=B, sigma=sigma, C1=C1, C2=C2, n=n, **{
        key: c[key] for key in ("m", "r", "k", "maxit", "tol", "p", "sketch_seed")})
    if "s" in c:  # the paper's fixed sketch size (kept as s_paper for the DCT embedding)
        out["s_paper"] = c["s"]
        s = max(c["s"], (c["maxit"] + 1) * c["r"])
    else:
        s = c["s_per"] * c["maxit"] * c["r"]
    out["s"] = -(-s // 8) * 8  # a multiple of the sparse-sign column count
    if "nu" in c:
        out["nu"] = c["nu"]
    out["zeta"] = 8
    if "loss_seed" in c:
        out["P1"] = gaussian_block(n, 4, c["loss_seed"])
        out["P2"] = gaussian_block(B.n, 4, c["loss_seed"] + 1000)
    return out
