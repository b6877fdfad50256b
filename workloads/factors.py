"""Seeded Gaussian blocks for right-hand sides and loss factors."""
from __future__ import annotations

import numpy as np


def gaussian_block(n: int, r: int, seed: int) -> np.ndarray:
    """An ``n x r`` block of i.i.d. N(0,1) entries from ``PCG64(seed)``, C-contiguous."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.ascontiguousarray(rng.standard_normal((n, r)))


def gaussian_factors(n1: int, n2: int, r: int, seed: int) -> tuple[np.ndarray, np.ndarray]:
    """Gaussian ``C1 (n1 x r)``, ``C2 (n2 x r)`` scaled so that ``||C1 C2^T||_F = 1``.

    Both factors are drawn from one ``PCG64(seed)`` stream (``C1`` first) and each is
    multiplied by ``||C1 C2^T||_F^(-1/2)``, mirroring the unit-norm right-hand sides of
    the paper's experiments (Sec. 6, Examples 6.1 and 6.3).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    C1 = rng.standard_normal((n1, r))
    C2 = rng.standard_normal((n2, r))
    nrm2 = float(np.sum((C1.T @ C1) * (C2.T @ C2)))  # ||C1 C2^T||_F^2 = tr((C1^T C1)(C2^T C2))
    f = nrm2 ** -0.25
    return np.ascontiguousarray(C1 * f), np.ascontiguousarray(C2 * f)
