"""Seeded synthetic inputs for the sketched-and-truncated Krylov Sylvester solver.

This package builds the *inputs* of a Sylvester equation ``A X + X B = C1 C2^T``:
sparse stencil operators in CSR form and Gaussian low-rank right-hand-side factors.
It holds none of the solver's arithmetic (no Krylov step, no sketch, no projected
solve), so both the FP64 test oracle and the GPU library may consume what it makes.

The operators are finite-difference discretisations of the PDE operators the paper
experiments with (convection-diffusion on the unit square and cube, Sec. 6,
Examples 6.1 and 6.3), with Gaussian right-hand sides normalised to unit Frobenius
norm as in those examples.
"""
from .stencil import (
    CSR,
    laplacian_2d,
    convdiff_2d_upwind,
    convdiff_centered,
    diffusion_3d,
    vardiff_2d,
    lognormal_field_2d,
    with_diag_shift,
)
from .factors import gaussian_factors, gaussian_block
from .configs import CONFIGS, make_config

__all__ = [
    "CSR",
    "laplacian_2d",
    "convdiff_2d_upwind",
    "convdiff_centered",
    "diffusion_3d",
    "vardiff_2d",
    "lognormal_field_2d",
    "with_diag_shift",
    "gaussian_factors",
    "gaussian_block",
    "CONFIGS",
    "make_config",
]
