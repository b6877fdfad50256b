"""Pins for the oracle's embeddings (Sec. 2.2: oblivious subspace embeddings)."""
import os

import numpy as np
import pytest

from oracle import sketch

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "splitmix64.txt")


def _golden():
    rows = []
    with open(GOLDEN) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                seed, idx, out = line.split()
                rows.append((int(seed), int(idx), int(out)))
    return rows


def test_splitmix64_known_answers():
    for seed, idx, out in _golden():
        assert sketch.splitmix64_stream(seed, idx)[-1] == out
        assert int(sketch.splitmix64_at(seed, np.array([idx]))[0]) == out


def test_sparse_sign_structure():
    n, s, zeta, seed = 500, 96, 8, 77
    rows, signs = sketch.sparse_sign_entries(n, s, zeta, seed)
    b = s // zeta
    # one nonzero per band, hence distinct rows within each column
    assert np.all(rows // b == np.arange(zeta)[None, :])
    assert np.all(np.abs(signs) == 1.0)
    S = sketch.sparse_sign(n, s, zeta, seed).toarray()
    assert np.allclose(np.linalg.norm(S, axis=0), 1.0, atol=0, rtol=1e-15)
    assert np.all((S != 0).sum(axis=0) == zeta)
    # entries re-derived from the scalar generator stream (independent code path)
    for j in (0, 1, 13, n - 1):
        stream = sketch.splitmix64_stream(seed, zeta * j + zeta)
        for t in range(zeta):
            z = stream[zeta * j + t]
            row = t * b + (((z >> 32) * b) >> 32)
            val = (-1.0 if z & 1 else 1.0) / np.sqrt(zeta)
            assert S[row, j] == val


def test_sparse_sign_is_subspace_embedding():
    """A random 20-dim subspace of R^4000 keeps its norms within a crude epsilon (s = 20*20)."""
    rng = np.random.Generator(np.random.PCG64(5))
    n, dim, s = 4000, 20, 400
    Qb, _ = np.linalg.qr(rng.standard_normal((n, dim)))
    S = sketch.sparse_sign(n, s, 8, 123)
    sv = np.linalg.svd(S @ Qb, compute_uv=False)
    assert sv.max() ** 2 < 1.5 and sv.min() ** 2 > 0.5


def test_space_seeds_differ():
    su, sv = sketch.space_seeds(42)
    assert su == 42 and sv == sketch.mix64_int(43) and su != sv


def test_srht_full_sampling_is_orthogonal():
    """With s = n every row is kept: S^T S = I (orthonormal DCT times signs)."""
    n = 64
    S = sketch.SRHT(n, n, 9).dense()
    assert np.allclose(S.T @ S, np.eye(n), atol=1e-13)


@pytest.mark.parametrize("n,s", [(7, 3), (12, 5), (15, 15)])
def test_srht_entries_match_the_dct_definition(n, s):
    """Brute force from the definitions: entry (i, j) of S = sqrt(n/s) D N E is
    sqrt(n/s) sqrt(2/n) c_k cos(pi k (2j+1) / (2n)) E_j with k = rows[i], c_0 = 1/sqrt(2),
    c_k = 1 otherwise (the orthonormal DCT-II); E_j is -1 exactly when output j+1 of SplitMix64
    from the seed is odd; rows are the s indices with the smallest outputs of the generator
    started at mix64(seed), ascending (a transposed N, signs applied after the transform, a
    wrong scale or a wrong draw all fail this)."""
    seed = 12345
    S = sketch.SRHT(n, s, seed).dense()
    outs = sketch.splitmix64_stream(seed, n)
    E = [-1.0 if z & 1 else 1.0 for z in outs]
    keys = sketch.splitmix64_stream(sketch.mix64_int(seed), n)
    rows = sorted(sorted(range(n), key=lambda i: (keys[i], i))[:s])
    ref = np.zeros((s, n))
    for i, k in enumerate(rows):
        ck = 1.0 / np.sqrt(2.0) if k == 0 else 1.0
        for j in range(n):
            ref[i, j] = np.sqrt(n / s) * np.sqrt(2.0 / n) * ck * np.cos(np.pi * k * (2 * j + 1) / (2 * n)) * E[j]
    assert np.abs(S - ref).max() < 1e-13


def test_srht_norm_preserved_in_expectation():
    n, s = 256, 64
    x = np.random.Generator(np.random.PCG64(3)).standard_normal(n)
    vals = [np.linalg.norm(sketch.SRHT(n, s, seed) @ x) ** 2 for seed in range(200)]
    assert abs(np.mean(vals) / np.dot(x, x) - 1.0) < 0.05


@pytest.mark.parametrize("kind", ["sparse_sign", "srht", "gaussian", "identity"])
def test_make_shapes(kind):
    n, s = 128, (128 if kind == "identity" else 32)
    S = sketch.make(kind, n, s, 8, 1)
    Y = S @ np.ones((n, 2))
    assert Y.shape == (s, 2)
