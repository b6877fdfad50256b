"""Finite-difference stencil operators on the unit square / cube, as CSR arrays.

Conventions (shared by every operator built here):

* homogeneous Dirichlet boundary, ``m`` interior nodes per direction, ``h = 1/(m+1)``;
* lexicographic ordering with ``x`` fastest: node ``(ix, iy)`` has index ``iy*m + ix``,
  node ``(ix, iy, iz)`` has index ``(iz*m + iy)*m + ix``;
* diffusion is scaled by ``1/h^2`` and convection by ``1/h``; every operator is the
  positive (``-Delta``-like) form, so its spectrum lies in the right half plane;
* first-order upwind convection: for ``w_c > 0`` the backward neighbour in direction
  ``c`` carries ``-|w_c|/h`` (forward neighbour for ``w_c < 0``) and the diagonal
  carries ``+|w_c|/h``;
* centered convection (``convdiff_centered``, the scheme of the paper's Sec. 6): the
  forward neighbour in direction ``c`` carries ``+w_c(x)/(2h)`` and the backward one
  ``-w_c(x)/(2h)``, with the velocity evaluated at the node.

The operators mirror the convection-diffusion workloads of the paper's experiments
(Sec. 6, Example 6.1 on the unit square and Example 6.3 on the unit cube):
``convdiff_centered`` builds those examples' operators; the upwind scheme and the
variable-coefficient diffusion of the other workloads are this package's choices.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp


@dataclass
class CSR:
    """A square sparse matrix in CSR form with int32 indices and float64 values."""

    n: int
    indptr: np.ndarray   # int32[n+1]
    indices: np.ndarray  # int32[nnz], sorted within each row
    data: np.ndarray     # float64[nnz]

    @property
    def nnz(self) -> int:
        return int(self.indptr[-1])

    def to_scipy(self) -> sp.csr_matrix:
        return sp.csr_matrix((self.data, self.indices, self.indptr), shape=(self.n, self.n))

    @staticmethod
    def from_scipy(M) -> "CSR":
        M = sp.csr_matrix(M)
        M.sum_duplicates()
        M.sort_indices()
        if M.shape[0] != M.shape[1]:
            raise ValueError("square matrices only")
        if M.nnz >= 2**31:
            raise ValueError("nnz exceeds int32 indexing")
        return CSR(
            n=M.shape[0],
            indptr=np.ascontiguousarray(M.indptr, dtype=np.int32),
            indices=np.ascontiguousarray(M.indices, dtype=np.int32),
            data=np.ascontiguousarray(M.data, dtype=np.float64),
        )

    def transpose(self) -> "CSR":
        return CSR.from_scipy(self.to_scipy().T.tocsr())


def _second_difference(m: int) -> sp.csr_matrix:
    """1D ``-d^2/dx^2`` with Dirichlet ends, scaled by ``1/h^2``."""
    h = 1.0 / (m + 1)
    e = np.ones(m)
    return sp.diags([-e[:-1], 2.0 * e, -e[:-1]], [-1, 0, 1], format="csr") / h**2


def _upwind_first_difference(m: int, w: float) -> sp.csr_matrix:
    """1D first-order upwind discretisation of ``w d/dx`` with Dirichlet ends."""
    h = 1.0 / (m + 1)
    e = np.ones(m)
    a = abs(w) / h
    if w >= 0.0:
        return sp.diags([-a * e[:-1], a * e], [-1, 0], format="csr")
    return sp.diags([a * e, -a * e[:-1]], [0, 1], format="csr")


def laplacian_2d(m: int) -> CSR:
    """5-point ``-Delta`` on an ``m x m`` interior grid (SPD, ``n = m^2``)."""
    I = sp.identity(m, format="csr")
    T = _second_difference(m)
    return CSR.from_scipy(sp.kron(I, T) + sp.kron(T, I))


def convdiff_2d_upwind(m: int, nu: float, w: tuple[float, float]) -> CSR:
    """5-point ``-nu Delta u + w . grad u`` with first-order upwind convection."""
    I = sp.identity(m, format="csr")
    T = _second_difference(m)
    Dx = _upwind_first_difference(m, w[0])
    Dy = _upwind_first_difference(m, w[1])
    M = nu * (sp.kron(I, T) + sp.kron(T, I)) + sp.kron(I, Dx) + sp.kron(Dy, I)
    return CSR.from_scipy(M)


def diffusion_3d(m: int, k: tuple[float, float, float] = (1.0, 1.0, 1.0), shift: float = 0.0) -> CSR:
    """7-point ``-(kx d_xx + ky d_yy + kz d_zz) + shift*I`` on an ``m^3`` interior grid."""
    I = sp.identity(m, format="csr")
    T = _second_difference(m)
    M = (
        k[0] * sp.kron(I, sp.kron(I, T))
        + k[1] * sp.kron(I, sp.kron(T, I))
        + k[2] * sp.kron(T, sp.kron(I, I))
    )
    if shift != 0.0:
        M = M + shift * sp.identity(m**3, format="csr")
    return CSR.from_scipy(M)


def vardiff_2d(kappa: np.ndarray) -> CSR:
    """5-point ``-div(kappa grad u)`` for a nodal coefficient field ``kappa[iy, ix]``.

    Interior faces take the harmonic mean of the two node values; a boundary face
    takes the value of its interior node.  The result is symmetric positive definite.
    """
    kappa = np.asarray(kappa, dtype=np.float64)
    m = kappa.shape[0]
    if kappa.shape != (m, m):
        raise ValueError("kappa must be square")
    h = 1.0 / (m + 1)
    idx = np.arange(m * m).reshape(m, m)
    # face coefficients between (iy, ix) and (iy, ix+1): shape (m, m-1)
    fx = 2.0 * kappa[:, :-1] * kappa[:, 1:] / (kappa[:, :-1] + kappa[:, 1:])
    fy = 2.0 * kappa[:-1, :] * kappa[1:, :] / (kappa[:-1, :] + kappa[1:, :])
    diag = np.zeros((m, m))
    diag[:, :-1] += fx
    diag[:, 1:] += fx
    diag[:-1, :] += fy
    diag[1:, :] += fy
    # boundary faces use the node value
    diag[:, 0] += kappa[:, 0]
    diag[:, -1] += kappa[:, -1]
    diag[0, :] += kappa[0, :]
    diag[-1, :] += kappa[-1, :]
    rows = [idx.ravel(), idx[:, :-1].ravel(), idx[:, 1:].ravel(), idx[:-1, :].ravel(), idx[1:, :].ravel()]
    cols = [idx.ravel(), idx[:, 1:].ravel(), idx[:, :-1].ravel(), idx[1:, :].ravel(), idx[:-1, :].ravel()]
    vals = [diag.ravel(), -fx.ravel(), -fx.ravel(), -fy.ravel(), -fy.ravel()]
    M = sp.coo_matrix(
        (np.concatenate(vals) / h**2, (np.concatenate(rows), np.concatenate(cols))), shape=(m * m, m * m)
    )
    return CSR.from_scipy(M.tocsr())


def lognormal_field_2d(m: int, corr_len: float, seed: int, pad: int = 2) -> np.ndarray:
    """``kappa = exp(g)`` with ``g`` a standardised Gaussian field on the interior nodes.

    ``g`` has squared-exponential covariance ``exp(-|x-y|^2 / (2 corr_len^2))``; it is
    sampled spectrally (white noise filtered by the square root of the spectral
    density) on a periodic grid ``pad`` times larger than the domain, cropped to the
    ``m x m`` interior nodes, then shifted/scaled to sample mean 0 and variance 1.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    N = pad * m
    h = 1.0 / (m + 1)
    kx = 2.0 * np.pi * np.fft.fftfreq(N, d=h)
    ky = 2.0 * np.pi * np.fft.rfftfreq(N, d=h)
    K2 = kx[:, None] ** 2 + ky[None, :] ** 2
    amp = np.exp(-0.25 * corr_len**2 * K2)  # sqrt of the SE spectral density (up to a constant)
    xi = rng.standard_normal((N, N))
    g = np.fft.irfft2(np.fft.rfft2(xi) * amp, s=(N, N))[:m, :m]
    g = (g - g.mean()) / g.std()
    return np.exp(g)


def convdiff_centered(m: int, dim: int, nu: float, wfun) -> CSR:
    """``-nu Delta u + w(x) . grad u`` by centered differences on an ``m^dim`` grid.

    ``wfun(*coords)`` returns the ``dim`` velocity components at the given node
    coordinates (arrays of the grid's shape, ``coords[0]`` = x).  Per direction ``c``
    the node's row gets ``2 nu / h^2`` on the diagonal and
    ``-nu / h^2 +- w_c / (2h)`` on the forward (+) and backward (-) neighbours; a
    neighbour outside the domain is a homogeneous Dirichlet value and drops out.
    """
    h = 1.0 / (m + 1)
    x = (np.arange(m) + 1) * h
    shape = (m,) * dim
    # grid arrays indexed [.., iz, iy, ix] so that ravel() is the x-fastest ordering
    grids = np.meshgrid(*([x] * dim), indexing="ij")[::-1]  # grids[c] varies along axis dim-1-c
    w = [np.broadcast_to(np.asarray(wc, dtype=np.float64), shape) for wc in wfun(*grids)]
    if len(w) != dim:
        raise ValueError("wfun must return one velocity component per direction")
    idx = np.arange(m**dim).reshape(shape)
    rows, cols, vals = [idx.ravel()], [idx.ravel()], [np.full(m**dim, 2.0 * dim * nu / h**2)]
    for c in range(dim):
        ax = dim - 1 - c  # the array axis of direction c
        lo = [slice(None)] * dim
        hi = [slice(None)] * dim
        lo[ax] = slice(0, m - 1)
        hi[ax] = slice(1, m)
        lo, hi = tuple(lo), tuple(hi)
        # forward neighbour of the nodes in `lo` is the node in `hi`, and vice versa
        rows += [idx[lo].ravel(), idx[hi].ravel()]
        cols += [idx[hi].ravel(), idx[lo].ravel()]
        vals += [-nu / h**2 + w[c][lo].ravel() / (2 * h), -nu / h**2 - w[c][hi].ravel() / (2 * h)]
    M = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(m**dim, m**dim))
    return CSR.from_scipy(M.tocsr())


def with_diag_shift(A: CSR, sigma: np.ndarray) -> CSR:
    """``A + diag(sigma)`` as a new CSR matrix."""
    sigma = np.asarray(sigma, dtype=np.float64)
    if sigma.shape != (A.n,):
        raise ValueError("sigma must have length n")
    return CSR.from_scipy(A.to_scipy() + sp.diags(sigma))
