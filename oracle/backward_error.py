"""Backward-error estimates for least squares -- oracle side (test infrastructure only).

Paper, Section 4.1 ("Quality assurance"):
  * BE_theta(x) = min ||[dA, theta db]||_F over perturbations making x the LS solution
    (eq:backward_error);
  * the Karlson-Walden estimate
        KW_theta(x) = theta / sqrt(1 + theta^2 ||x||^2)
                      * || (A^T A + lambda I)^{-1/2} A^T r ||,
        lambda = theta^2 ||r||^2 / (1 + theta^2 ||x||^2),  r = b - A x,
    with KW <= BE <= sqrt(2) KW (Fact 4.1);
  * the sketched estimate (eq:sketched-kw) with (S A)^T (S A) in place of A^T A, evaluated from
    the SVD S A = U Sigma V^T as theta / sqrt(1 + theta^2 ||x||^2) * ||(Sigma^2 + lambda I)^{-1/2}
    V^T A^T r|| (the closing display of Section 4.1); bounded by Proposition 4.2.
The exact BE is only cited by the paper (the Walden-Karlson-Sun formula, as presented in
Higham's "Accuracy and Stability of Numerical Algorithms", Theorem 20.5):
    mu = theta^2 ||x||^2 / (1 + theta^2 ||x||^2),  phi = sqrt(mu) ||r|| / ||x||,
    BE = min(phi, sigma_min([A, phi (I - r r^T / ||r||^2)])),
(equivalently BE^2 = phi^2 + min(0, lambda_min(A A^T - phi^2 r r^T / ||r||^2)), but the
singular-value form avoids the cancellation of the squared form).  O(m^3); used on tiny inputs
only and pinned through Fact 4.1.
"""

from __future__ import annotations

import numpy as np


def _lambda(theta, rnorm, xnorm):
    if np.isinf(theta):
        return rnorm**2 / xnorm**2, 1.0 / xnorm
    return (theta**2 * rnorm**2) / (1.0 + theta**2 * xnorm**2), theta / np.sqrt(1.0 + theta**2 * xnorm**2)


def kw_from_svd(sigma, V, g, theta, rnorm, xnorm):
    """theta/sqrt(1+theta^2||x||^2) * ||(Sigma^2 + lambda)^{-1/2} V^T g|| for any (Sigma, V)."""
    lam, pref = _lambda(theta, rnorm, xnorm)
    w = V.T @ g
    return pref * np.sqrt(np.sum(w * w / (sigma**2 + lam)))


def kw_estimate(A, b, x, theta):
    """Karlson-Walden estimate via the SVD of A (Section 4.1).  O(m n^2)."""
    r = b - A @ x
    _, s, Vt = np.linalg.svd(A, full_matrices=False)
    return kw_from_svd(s, Vt.T, A.T @ r, theta, np.linalg.norm(r), np.linalg.norm(x))


def kw_estimate_dense(A, b, x, theta):
    """The same estimate written literally: the matrix (A^T A + lambda I)^{-1/2} via eigh (tiny n)."""
    r = b - A @ x
    lam, pref = _lambda(theta, np.linalg.norm(r), np.linalg.norm(x))
    M = A.T @ A + lam * np.eye(A.shape[1])
    w, Q = np.linalg.eigh(M)
    Minvhalf = (Q / np.sqrt(w)) @ Q.T
    return pref * np.linalg.norm(Minvhalf @ (A.T @ r))


def kw_known_svd(A, b, x, sigma, V, theta, accurate=True):
    """KW for a generated problem A = U diag(sigma) V^T whose SVD is known.  O(m n).

    ``g = A^T r`` is formed from the stored A; with ``accurate`` the residual and the product are
    accumulated in extended precision (numpy longdouble).
    """
    if accurate:
        xl = np.asarray(x, dtype=np.longdouble)
        g = np.zeros(A.shape[1], dtype=np.longdouble)
        rr = np.longdouble(0.0)
        for i0 in range(0, A.shape[0], 8192):
            Al = np.asarray(A[i0:i0 + 8192], dtype=np.longdouble)
            r = np.asarray(b[i0:i0 + 8192], dtype=np.longdouble) - Al @ xl
            g += Al.T @ r
            rr += np.sum(r * r)
        g = np.asarray(g, dtype=np.float64)
        rn = float(np.sqrt(rr))
    else:
        r = b - A @ x
        g = A.T @ r
        rn = np.linalg.norm(r)
    return kw_from_svd(sigma, V, g, theta, rn, np.linalg.norm(x))


def sketched_kw(A, b, x, sigma_sk, V_sk, theta):
    """Sketched KW (eq:sketched-kw) from the SVD of the sketch S A = U Sigma V^T."""
    r = b - A @ x
    return kw_from_svd(sigma_sk, V_sk, A.T @ r, theta, np.linalg.norm(r), np.linalg.norm(x))


def exact_backward_error(A, b, x, theta):
    """Walden-Karlson-Sun backward error BE_theta(x) (eq:backward_error).  O(m^3); tiny m only."""
    r = b - A @ x
    rn = np.linalg.norm(r)
    xn = np.linalg.norm(x)
    if xn == 0.0:
        raise ValueError("exact backward error defined here for x != 0")
    if rn == 0.0:
        return 0.0
    mu = 1.0 if np.isinf(theta) else theta**2 * xn**2 / (1.0 + theta**2 * xn**2)
    phi = np.sqrt(mu) * rn / xn
    m = A.shape[0]
    B = np.concatenate([A, phi * (np.eye(m) - np.outer(r, r) / rn**2)], axis=1)   # m x (n + m)
    smin = np.linalg.svd(B, compute_uv=False)[m - 1]
    return float(min(phi, smin))


def relative_backward_error(A, b, x, sigma=None, V=None):
    """Relative BE estimate KW_theta(x) / ||A||_F with theta = ||A||_F / ||b|| (Alg 4's choice).

    Uses the known SVD when (sigma, V) are given, else the SVD of A.
    """
    fro = np.linalg.norm(A)
    theta = fro / np.linalg.norm(b)
    if sigma is not None:
        return kw_known_svd(A, b, x, sigma, V, theta) / fro
    return kw_estimate(A, b, x, theta) / fro


# ---------------------------------------------------------------- complex problems
# The same estimate over C (Section 4.1's formula with conjugate transposes):
#   KW_theta(x) = theta / sqrt(1 + theta^2 ||x||^2) * || (A^H A + lambda I)^{-1/2} A^H r ||,
# evaluated from an SVD A = U diag(sigma) V^H as ||diag((sigma^2 + lambda)^{-1/2}) V^H A^H r||.


def kw_complex(A, b, x, theta, sigma=None, V=None):
    """Complex KW; g = A^H r and ||r|| accumulated in extended precision (numpy clongdouble)."""
    xl = np.asarray(x, dtype=np.clongdouble)
    g = np.zeros(A.shape[1], dtype=np.clongdouble)
    rr = np.longdouble(0.0)
    for i0 in range(0, A.shape[0], 8192):
        Al = np.asarray(A[i0:i0 + 8192], dtype=np.clongdouble)
        r = np.asarray(b[i0:i0 + 8192], dtype=np.clongdouble) - Al @ xl
        g += Al.conj().T @ r
        rr += np.sum(np.abs(r) ** 2)
    g = np.asarray(g, dtype=np.complex128)
    if sigma is None:
        _, sigma, Vh = np.linalg.svd(A, full_matrices=False)
        V = Vh.conj().T
    lam, pref = _lambda(theta, float(np.sqrt(rr)), np.linalg.norm(x))
    w = V.conj().T @ g
    return pref * np.sqrt(np.sum(np.abs(w) ** 2 / (sigma**2 + lam)))


def relative_backward_error_complex(A, b, x, sigma=None, V=None):
    """KW_theta(x) / ||A||_F with theta = ||A||_F / ||b|| for complex A, b, x."""
    fro = np.linalg.norm(A)
    theta = fro / np.linalg.norm(b)
    return kw_complex(A, b, x, theta, sigma, V) / fro
