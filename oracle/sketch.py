"""Oblivious subspace embeddings ``S`` (Sec. 2.2 of the paper), FP64, materialised.

The sparse sign embedding (the embedding the GPU path applies) is defined here from
its description, independently of any GPU code:

* ``s`` is a multiple of ``zeta`` and ``b = s / zeta``;
* column ``j`` of ``S`` has exactly ``zeta`` nonzeros, one in each row band
  ``[t*b, (t+1)*b)`` for ``t = 0..zeta-1``;
* the copy ``(j, t)`` draws ``z = splitmix64_output(seed, zeta*j + t + 1)``, i.e. the
  ``(zeta*j+t+1)``-th output of the SplitMix64 generator started at state ``seed``
  (Steele, Lea and Flood, OOPSLA 2014): ``z = mix64(seed + i*0x9E3779B97F4A7C15)``;
* the row is ``t*b + floor(hi32(z) * b / 2^32)`` and the value is ``-1/sqrt(zeta)`` when
  the lowest bit of ``z`` is set, else ``+1/sqrt(zeta)``.

Every column therefore has unit Euclidean norm.  The two spaces of the method use
independent embeddings (Algorithm 1 takes ``S_U`` and ``S_V`` as inputs): ``S_U``
uses ``seed`` and ``S_V`` uses ``mix64(seed + 1)``.

The subsampled trigonometric transform of Sec. 6, ``S = c * D N E`` with a Rademacher
diagonal ``E``, the orthonormal DCT-II ``N`` and ``s`` distinct sampled rows ``D``, is
provided with ``c = sqrt(n/s)`` (the paper prints ``sqrt(s/n)``; with an orthonormal
DCT only ``sqrt(n/s)`` preserves norms in expectation, and the computed solution does
not depend on a scalar factor in ``S``).
"""
from __future__ import annotations

import numpy as np
import scipy.fft
import scipy.sparse as sp

GOLDEN_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_MASK = (1 << 64) - 1


def mix64_int(z: int) -> int:
    """SplitMix64 output function on a Python int (reference scalar version)."""
    z &= _MASK
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK
    return z ^ (z >> 31)


def splitmix64_stream(seed: int, count: int) -> list[int]:
    """The first ``count`` outputs of SplitMix64 started at state ``seed``."""
    out, state = [], seed & _MASK
    for _ in range(count):
        state = (state + 0x9E3779B97F4A7C15) & _MASK
        out.append(mix64_int(state))
    return out


def mix64(z: np.ndarray) -> np.ndarray:
    """Vectorised SplitMix64 output function on uint64 arrays (wrap-around arithmetic)."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def splitmix64_at(seed: int, index: np.ndarray) -> np.ndarray:
    """Output number ``index`` (1-based) of SplitMix64 started at ``seed``."""
    index = np.asarray(index, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return mix64(np.uint64(seed & _MASK) + index * GOLDEN_GAMMA)


def space_seeds(seed: int) -> tuple[int, int]:
    """Seeds of ``S_U`` and ``S_V`` derived from one user seed."""
    return seed & _MASK, mix64_int((seed + 1) & _MASK)


def sparse_sign_entries(n: int, s: int, zeta: int, seed: int) -> tuple[np.ndarray, np.ndarray]:
    """Rows ``(n, zeta)`` int64 and signs ``(n, zeta)`` float64 (+-1) of the sparse sign map."""
    if s % zeta != 0:
        raise ValueError("s must be a multiple of zeta")
    b = s // zeta
    j = np.arange(n, dtype=np.uint64)[:, None]
    t = np.arange(zeta, dtype=np.uint64)[None, :]
    z = splitmix64_at(seed, np.uint64(zeta) * j + t + np.uint64(1))
    hi = z >> np.uint64(32)
    bucket = (hi * np.uint64(b)) >> np.uint64(32)  # floor(hi * b / 2^32) < b
    rows = t.astype(np.int64) * b + bucket.astype(np.int64)
    signs = np.where((z & np.uint64(1)) != 0, -1.0, 1.0)
    return rows, signs


def sparse_sign(n: int, s: int, zeta: int, seed: int) -> sp.csr_matrix:
    """The ``s x n`` sparse sign embedding as a SciPy CSR matrix."""
    rows, signs = sparse_sign_entries(n, s, zeta, seed)
    cols = np.repeat(np.arange(n, dtype=np.int64), zeta)
    vals = signs.ravel() / np.sqrt(zeta)
    return sp.csr_matrix((vals, (rows.ravel(), cols)), shape=(s, n))


class SRHT:
    """Subsampled randomized DCT ``S x = sqrt(n/s) * DCT2_ortho(E x)[rows]`` (Sec. 6).

    ``E_j = -1`` when the lowest bit of ``splitmix64_at(seed, j+1)`` is set, else +1;
    ``rows`` are the ``s`` indices with the smallest ``splitmix64_at(mix64(seed), i+1)``
    keys, in ascending index order (sampling without replacement).
    """

    def __init__(self, n: int, s: int, seed: int):
        if not 0 < s <= n:
            raise ValueError("need 0 < s <= n")
        self.n, self.s = n, s
        idx = np.arange(1, n + 1, dtype=np.uint64)
        self.E = np.where((splitmix64_at(seed, idx) & np.uint64(1)) != 0, -1.0, 1.0)
        keys = splitmix64_at(mix64_int(seed), idx)
        self.rows = np.sort(np.argsort(keys, kind="stable")[:s])
        self.scale = np.sqrt(n / s)

    def __matmul__(self, X: np.ndarray) -> np.ndarray:
        X = np.asarray(X, dtype=np.float64)
        vec = X.ndim == 1
        X2 = X[:, None] if vec else X
        Y = scipy.fft.dct(self.E[:, None] * X2, type=2, norm="ortho", axis=0)[self.rows] * self.scale
        return Y[:, 0] if vec else Y

    def dense(self) -> np.ndarray:
        return self @ np.eye(self.n)


def gaussian(n: int, s: int, seed: int) -> np.ndarray:
    """Dense Gaussian embedding with ``N(0, 1/s)`` entries (footnote of Sec. 2.2)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal((s, n)) / np.sqrt(s)


def make(kind: str, n: int, s: int, zeta: int, seed: int):
    """Build ``S`` of the requested kind: ``'sparse_sign'``, ``'srht'``, ``'gaussian'`` or ``'identity'``."""
    if kind == "sparse_sign":
        return sparse_sign(n, s, zeta, seed)
    if kind == "srht":
        return SRHT(n, s, seed)
    if kind == "gaussian":
        return gaussian(n, s, seed)
    if kind == "identity":
        return sp.identity(n, format="csr")
    raise ValueError(kind)
