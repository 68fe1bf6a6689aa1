"""Pins for the oracle's Householder QR least-squares solver (CPU only)."""

from fractions import Fraction

import numpy as np
import pytest

from oracle import householder as hh

U = 2.0**-52


def _normal_equations_longdouble(A, b):
    Al = np.asarray(A, dtype=np.longdouble)
    bl = np.asarray(b, dtype=np.longdouble)
    G = Al.T @ Al
    h = Al.T @ bl
    n = G.shape[0]
    # Gaussian elimination with partial pivoting in long double
    M = np.concatenate([G, h[:, None]], axis=1)
    for k in range(n):
        p = k + int(np.argmax(np.abs(M[k:, k])))
        M[[k, p]] = M[[p, k]]
        for i in range(k + 1, n):
            M[i] -= M[i, k] / M[k, k] * M[k]
    x = np.zeros(n, dtype=np.longdouble)
    for i in range(n - 1, -1, -1):
        x[i] = (M[i, n] - M[i, i + 1:n] @ x[i + 1:]) / M[i, i]
    return x.astype(np.float64)


@pytest.mark.parametrize("seed", range(5))
def test_qr_ls_matches_extended_normal_equations(seed):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((8, 3))
    b = rng.standard_normal(8)
    x = hh.qr_lstsq(A, b)
    xr = _normal_equations_longdouble(A, b)
    assert np.max(np.abs(x - xr)) <= 50 * U * np.linalg.cond(A) ** 2 * np.linalg.norm(xr) + 1e-14


def _rational_lstsq(A, b):
    n = len(A[0])
    G = [[sum(Fraction(A[k][i]) * A[k][j] for k in range(len(A))) for j in range(n)] for i in range(n)]
    h = [sum(Fraction(A[k][i]) * b[k] for k in range(len(A))) for i in range(n)]
    for k in range(n):
        p = next(i for i in range(k, n) if G[i][k] != 0)
        G[k], G[p], h[k], h[p] = G[p], G[k], h[p], h[k]
        for i in range(k + 1, n):
            f = G[i][k] / G[k][k]
            G[i] = [G[i][j] - f * G[k][j] for j in range(n)]
            h[i] -= f * h[k]
    x = [Fraction(0)] * n
    for i in range(n - 1, -1, -1):
        x[i] = (h[i] - sum(G[i][j] * x[j] for j in range(i + 1, n))) / G[i][i]
    return x


def test_qr_ls_exact_rational_integer_system():
    rng = np.random.default_rng(42)
    A = rng.integers(-5, 6, size=(9, 4)).tolist()
    b = rng.integers(-9, 10, size=9).tolist()
    xe = np.array([float(v) for v in _rational_lstsq(A, b)])
    x = hh.qr_lstsq(np.array(A, dtype=float), np.array(b, dtype=float))
    assert np.max(np.abs(x - xe)) <= 1e-13 * max(1.0, np.max(np.abs(xe)))


def test_single_column_closed_form():
    rng = np.random.default_rng(3)
    a = rng.standard_normal((50, 1))
    b = rng.standard_normal(50)
    x = hh.qr_lstsq(a, b)
    assert abs(x[0] - (a[:, 0] @ b) / (a[:, 0] @ a[:, 0])) <= 1e-14 * abs(x[0])


def test_orthonormal_columns_give_projection():
    rng = np.random.default_rng(4)
    Q, _ = np.linalg.qr(rng.standard_normal((40, 6)))
    b = rng.standard_normal(40)
    assert np.allclose(hh.qr_lstsq(Q, b), Q.T @ b, rtol=0, atol=1e-14)


def test_factorization_residual_and_orthogonality():
    rng = np.random.default_rng(5)
    A = rng.standard_normal((60, 12)) @ np.diag(10.0 ** -np.arange(12))
    Qinfo, R = hh.householder_qr(A)
    assert np.all(np.diag(R) >= 0)
    Qt = np.stack([hh.apply_qt(Qinfo, e) for e in np.eye(60)], axis=1)   # Q^T, 60 x 60
    assert np.linalg.norm(Qt @ Qt.T - np.eye(60)) <= 60 * U * 10
    QtA = Qt @ A
    assert np.linalg.norm(QtA[:12] - R) <= 60 * U * np.linalg.norm(A) * 10
    assert np.linalg.norm(QtA[12:]) <= 60 * U * np.linalg.norm(A) * 10


def test_matches_lapack_lstsq_on_ill_conditioned_problem():
    from synth import make_problem
    P = make_problem(300, 20, 1e8, 1e-4, seed=1)
    x = hh.qr_lstsq(P.A, P.b)
    xl = np.linalg.lstsq(P.A, P.b, rcond=None)[0]
    # both backward stable: forward errors agree within the Wedin scale kappa^2 ||r|| u + kappa u ||x||
    scale = 1e8 * np.linalg.norm(P.x_true) * U + 1e16 * 1e-4 * U
    assert np.linalg.norm(x - xl) <= 20 * scale


def test_triangular_solvers():
    rng = np.random.default_rng(6)
    R = np.triu(rng.standard_normal((9, 9))) + 5 * np.eye(9)
    y = rng.standard_normal(9)
    assert np.allclose(R @ hh.back_substitution(R, y), y, atol=1e-13)
    assert np.allclose(R.T @ hh.forward_substitution_transposed(R, y), y, atol=1e-13)


# ---------------------------------------------------------------- TSQR reference (large problems)

def test_tsqr_exact_rational_integer_system():
    """A tree of three levels (block_rows small) on an integer system: the exact rational LS
    solution (normal equations in Fractions) to rounding."""
    rng = np.random.default_rng(7)
    A = rng.integers(-9, 10, size=(90, 4)).astype(float)
    b = rng.integers(-9, 10, size=90).astype(float)
    xr = np.array([float(v) for v in _rational_lstsq(A.tolist(), b.tolist())])
    x = hh.qr_lstsq_tsqr(A, b, block_rows=10, workers=3)
    assert np.max(np.abs(x - xr)) <= 1e3 * U * np.linalg.cond(A) * np.linalg.norm(xr)


def test_tsqr_special_cases():
    rng = np.random.default_rng(8)
    a = rng.standard_normal(500)
    b = rng.standard_normal(500)
    x = hh.qr_lstsq_tsqr(a[:, None], b, block_rows=40)
    assert abs(x[0] - (a @ b) / (a @ a)) <= 20 * U * abs(x[0])
    Q = np.linalg.qr(rng.standard_normal((400, 6)))[0]
    x = hh.qr_lstsq_tsqr(Q, b[:400], block_rows=30)
    assert np.linalg.norm(x - Q.T @ b[:400]) <= 100 * U * np.linalg.norm(b[:400])


def test_tsqr_triangle_reproduces_gram_matrix():
    """R of the stacked tree satisfies R^T R = M^T M to the backward error of Householder QR."""
    rng = np.random.default_rng(9)
    M = rng.standard_normal((700, 9)) @ np.diag(10.0 ** -np.arange(9))
    R = hh._tsqr_r(lambda i0, i1: M[i0:i1], 700, 9, 40, 4)
    assert np.allclose(R, np.triu(R))
    assert np.linalg.norm(R.T @ R - M.T @ M) <= 700 * U * np.linalg.norm(M) ** 2
    # singular values are those of M (QR is an orthogonal reduction)
    assert np.allclose(np.linalg.svd(R, compute_uv=False), np.linalg.svd(M, compute_uv=False), rtol=1e-10, atol=0)


def test_tsqr_matches_plain_householder_and_multi_rhs():
    """On an ill-conditioned problem the blocked reference and the plain loop agree within the
    Wedin scale; several right-hand sides give each column's single solve."""
    from synth import make_problem
    P = make_problem(3000, 25, 1e9, 1e-5, seed=2)
    x = hh.qr_lstsq(P.A, P.b)
    xt = hh.qr_lstsq_tsqr(P.A, P.b, block_rows=200, workers=4)
    scale = 1e9 * np.linalg.norm(P.x_true) * U + 1e18 * 1e-5 * U
    assert np.linalg.norm(x - xt) <= 20 * scale
    B = np.column_stack([P.b, 2.0 * P.b, P.A @ P.x_true])
    X = hh.qr_lstsq_tsqr(P.A, B, block_rows=200, workers=4)
    for j in range(3):
        assert np.linalg.norm(X[:, j] - hh.qr_lstsq_tsqr(P.A, B[:, j], block_rows=200)) <= 20 * scale * (1 + j)
    # consistent right-hand side: forward error at the kappa u level
    assert np.linalg.norm(X[:, 2] - P.x_true) <= 100 * 1e9 * U * np.linalg.norm(P.x_true)
