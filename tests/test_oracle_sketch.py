"""Pins for the oracle's sparse sign embedding (CPU only)."""

import numpy as np

from oracle import sketch
from synth import make_problem


def test_sparse_matches_dense_reference():
    rng = np.random.default_rng(0)
    m, n, d, zeta = 200, 7, 40, 5
    A = rng.standard_normal((m, n))
    Sd = sketch.dense_sign_matrix(m, d, zeta, 99)
    Y = sketch.sketch(A, d, zeta, 99)
    ref = (np.asarray(Sd, dtype=np.longdouble) @ np.asarray(A, dtype=np.longdouble)).astype(np.float64)
    assert np.max(np.abs(Y - ref)) <= 1e-14 * np.max(np.abs(ref))


def test_columns_of_S_have_unit_norm_and_zeta_nonzeros():
    Sd = sketch.dense_sign_matrix(300, 50, 8, 5)
    assert np.all(np.count_nonzero(Sd, axis=0) == 8)
    assert np.allclose(np.sum(Sd * Sd, axis=0), 1.0, rtol=0, atol=4e-16)


def test_expected_gram_is_identity():
    """E[S^T S] = I: diagonal is exactly 1; off-diagonal entries average to ~0 over the draw."""
    m, d = 400, 60
    Sd = sketch.dense_sign_matrix(m, d, 8, 11)
    G = Sd.T @ Sd
    off = G[~np.eye(m, dtype=bool)]
    assert abs(off.mean()) < 5e-3
    # Var of an off-diagonal entry: zeta^2 * (1/d) / zeta^2 ... ~ zeta/d/zeta = 1/d
    assert abs(off.var() - 1.0 / d) < 0.25 / d


def test_subspace_embedding_distortion():
    """Definition 2.1: the distortion of S on range(A) is near sqrt(n/d) for d = 12 n."""
    P = make_problem(4000, 50, 1e6, 1e-6, seed=3)
    Q, _ = np.linalg.qr(P.A)
    SQ = sketch.sketch(Q, 600, 8, 12345)
    s = np.linalg.svd(SQ, compute_uv=False)
    eta = max(s[0] - 1.0, 1.0 - s[-1])
    assert 0.15 < eta < 1.5 * np.sqrt(50 / 600)


def test_sketch_Ab_is_one_embedding():
    rng = np.random.default_rng(1)
    A, b = rng.standard_normal((500, 4)), rng.standard_normal(500)
    Y = sketch.sketch_Ab(A, b, 30, 8, 5)
    assert np.allclose(Y[:, :4], sketch.sketch(A, 30, 8, 5), rtol=0, atol=0)
    assert np.allclose(Y[:, 4], sketch.sketch(b, 30, 8, 5), rtol=0, atol=0)
