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
}

NU_CONVDIFF = 1e-2
W_A = (1.0, 0.5)
W_B = (-0.3, 1.0)
ANISO = (1.0, 10.0, 100.0)
CORR_LEN = 0.1


def make_config(name: str, m: int | None = None, maxit: int | None = None, r: int | None = None) -> dict:
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
    s = c["s_per"] * c["maxit"] * c["r"]
    out["s"] = -(-s // 8) * 8  # a multiple of the sparse-sign column count
    out["zeta"] = 8
    if "loss_seed" in c:
        out["P1"] = gaussian_block(n, 4, c["loss_seed"])
        out["P2"] = gaussian_block(B.n, 4, c["loss_seed"] + 1000)
    return out
