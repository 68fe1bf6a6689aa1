"""Oracle pins for the complex-valued problems (the Prony workload of Section 5.2, Appendix B).

The complex Householder least-squares solver is pinned by special cases that reduce to something
else (real input -> the real Householder solver; orthonormal columns -> x = A^H b; tiny systems ->
the normal equations in extended precision) and by its factorization; the complex KW estimate by
the realification identity against the real estimate and by its zero at the LS solution; the
Prony generator by Prony's method itself (noise-free samples: the least-squares prediction
coefficients are those of the polynomial with roots z_k, Appendix B's algorithm); complex FOSSILS
and SPIR by the backward-error bar.
"""

import numpy as np
import pytest

from oracle import backward_error as be
from oracle import householder as hh
from oracle import solvers
from synth import make_complex_problem, make_prony_problem, prony_samples

U = 2.0**-52


def test_complex_qr_of_real_input_is_the_real_solver():
    rng = np.random.default_rng(0)
    A = rng.standard_normal((60, 7)) * rng.uniform(0.1, 10, 7)
    b = rng.standard_normal(60)
    xc = hh.qr_lstsq_complex(A.astype(np.complex128), b.astype(np.complex128))
    xr = hh.qr_lstsq(A, b)
    assert np.max(np.abs(xc.imag)) == 0.0
    assert np.linalg.norm(xc.real - xr) <= 1e-14 * np.linalg.norm(xr)


def test_complex_qr_orthonormal_columns():
    P = make_complex_problem(300, 9, 1.0, 0.3, seed=1)   # sigma = 1: A = U V^H has orthonormal columns
    x = hh.qr_lstsq_complex(P.A, P.b)
    assert np.linalg.norm(x - P.A.conj().T @ P.b) <= 50 * U * np.linalg.norm(x)


def test_complex_qr_normal_equations_tiny():
    rng = np.random.default_rng(2)
    A = rng.standard_normal((8, 3)) + 1j * rng.standard_normal((8, 3))
    b = rng.standard_normal(8) + 1j * rng.standard_normal(8)
    Al, bl = A.astype(np.clongdouble), b.astype(np.clongdouble)
    G = Al.conj().T @ Al
    rhs = Al.conj().T @ bl
    # Gaussian elimination on the 3 x 3 Hermitian system in extended precision
    M = np.concatenate([G, rhs[:, None]], axis=1)
    for k in range(3):
        M[k] = M[k] / M[k, k]
        for i in range(3):
            if i != k:
                M[i] = M[i] - M[i, k] * M[k]
    xn = np.asarray(M[:, 3], dtype=np.complex128)
    x = hh.qr_lstsq_complex(A, b)
    assert np.linalg.norm(x - xn) <= 1e-13 * np.linalg.norm(xn)


def test_complex_qr_factorization():
    rng = np.random.default_rng(3)
    A = rng.standard_normal((40, 6)) + 1j * rng.standard_normal((40, 6))
    Q, R = hh.householder_qr_complex(A)
    d = np.diag(R)
    assert np.all(d.imag == 0) and np.all(d.real >= 0)
    QhA = np.stack([hh.apply_qh_complex(Q, A[:, j]) for j in range(6)], axis=1)
    assert np.linalg.norm(QhA[:6] - R) <= 50 * U * np.linalg.norm(A)
    assert np.linalg.norm(QhA[6:]) <= 50 * U * np.linalg.norm(A)
    # Q^H preserves norms
    y = rng.standard_normal(40) + 1j * rng.standard_normal(40)
    assert abs(np.linalg.norm(hh.apply_qh_complex(Q, y)) - np.linalg.norm(y)) <= 50 * U * np.linalg.norm(y)


def test_realification_is_an_isometry():
    P = make_complex_problem(200, 7, 1e4, 1e-2, seed=4)
    Ar, br = solvers.realify(P.A, P.b)
    rng = np.random.default_rng(5)
    z = rng.standard_normal(7) + 1j * rng.standard_normal(7)
    zr = np.concatenate([z.real, z.imag])
    assert abs(np.linalg.norm(Ar @ zr - br) - np.linalg.norm(P.A @ z - P.b)) <= 1e-13 * np.linalg.norm(P.b)
    s = np.linalg.svd(Ar, compute_uv=False)
    assert np.allclose(np.sort(s)[::-1], np.repeat(P.sigma, 2), rtol=1e-10, atol=0)


def test_complex_kw_equals_the_real_kw_of_the_realification():
    P = make_complex_problem(400, 8, 1e6, 1e-3, seed=6)
    rng = np.random.default_rng(7)
    x = P.x_true + 1e-9 * (rng.standard_normal(8) + 1j * rng.standard_normal(8))
    Ar, br = solvers.realify(P.A, P.b)
    xr = np.concatenate([x.real, x.imag])
    fro = np.linalg.norm(P.A)
    theta = fro / np.linalg.norm(P.b)
    kc = be.kw_complex(P.A, P.b, x, theta, P.sigma, P.V)
    kr = be.kw_estimate(Ar, br, xr, theta)
    assert abs(kc - kr) <= 1e-8 * kr
    # and without the known SVD
    assert abs(be.kw_complex(P.A, P.b, x, theta) - kr) <= 1e-8 * kr


def test_complex_kw_vanishes_at_the_ls_solution():
    P = make_complex_problem(300, 6, 1e3, 1e-2, seed=8)
    xq = hh.qr_lstsq_complex(P.A, P.b)
    assert be.relative_backward_error_complex(P.A, P.b, xq, P.sigma, P.V) <= 1e-15
    assert be.relative_backward_error_complex(P.A, P.b, P.x_true + 1e-6, P.sigma, P.V) >= 1e-9


def test_prony_generator_recovers_the_exponentials():
    """Noise-free samples of K = n exponentials: the least-squares prediction coefficients p give
    z^n - p_1 z^{n-1} - ... - p_n with roots z_k (Appendix B, lines 1-3 of Prony's method)."""
    n = 6
    P = make_prony_problem(200, n, n, noise=0.0, seed=9)
    x = hh.qr_lstsq_complex(P.A, P.b)
    assert np.linalg.norm(P.b - P.A @ x) <= 1e-10 * np.linalg.norm(P.b)
    roots = np.roots(np.concatenate([[1.0], -x]))
    z = P.meta["z"]
    for zk in z:
        assert np.min(np.abs(roots - zk)) <= 1e-6
    # Toeplitz structure: A[i, j] = f_{n-1+i-j}, b_i = f_{n-1+i} (0-based i, j)
    f, _, _ = prony_samples(200 + n, n, 0.0, 9)
    assert P.A[5, 2] == f[n - 1 + 5 - 2] and P.b[5] == f[n + 5]


@pytest.mark.parametrize("method", ["fossils", "spir"])
@pytest.mark.parametrize("kappa,rnorm", [(1e2, 1.0), (1e6, 1e-4), (1e10, 1e-8)])
def test_complex_fossils_oracle_meets_the_bar(method, kappa, rnorm):
    P = make_complex_problem(1500, 20, kappa, rnorm, seed=10)
    r = solvers.solve_complex(P.A, P.b, method, solvers.Options(precond="svd"))
    assert r.flags == 0
    assert be.relative_backward_error_complex(P.A, P.b, r.x, P.sigma, P.V) <= 1e-14
    xq = hh.qr_lstsq_complex(P.A, P.b)
    fe = np.linalg.norm(r.x - P.x_true) / np.linalg.norm(P.x_true)
    fq = max(np.linalg.norm(xq - P.x_true) / np.linalg.norm(P.x_true), kappa * U)
    assert fe <= 10 * fq


def test_complex_fossils_oracle_on_a_prony_problem():
    P = make_prony_problem(3000, 30, 10, 1e-6, seed=11)
    r = solvers.solve_complex(P.A, P.b, "fossils", solvers.Options(precond="svd"))
    assert r.flags == 0
    assert be.relative_backward_error_complex(P.A, P.b, r.x) <= 1e-14
    xq = hh.qr_lstsq_complex(P.A, P.b)
    assert np.linalg.norm(r.x - xq) <= 10 * r.condest * U * np.linalg.norm(xq)
