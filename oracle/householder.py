"""Householder QR and the QR least-squares solver -- oracle side (test infrastructure only).

The paper's classical baseline (Section 1: Householder QR is backward stable for least squares)
and the factorization its sketching analysis assumes for the sketch (Lemma 6.3, "computed using
Householder QR"; Section 6 states that triangular solves are back substitutions).

Textbook column-by-column Householder QR (no blocking): for column k, the reflector
H_k = I - 2 v v^T / (v^T v) with v = x + sign(x_0) ||x|| e_1 maps x = A[k:, k] to
-sign(x_0) ||x|| e_1 and is applied to the trailing columns.
"""

from __future__ import annotations

import numpy as np


def householder_qr(M: np.ndarray, positive_diag: bool = True):
    """Return (V, R) with the reflectors stored as a list of (k, v) and R upper triangular (k x k).

    ``M`` is m x k with m >= k; it is copied.  With ``positive_diag`` rows of R are negated so
    that diag(R) >= 0 (the implicit Q's columns are negated accordingly); the QR factorization
    itself is unchanged.
    """
    A = np.array(M, dtype=np.float64, order="F", copy=True)
    m, k = A.shape
    if m < k:
        raise ValueError("householder_qr expects m >= k")
    refl = []
    for j in range(k):
        x = A[j:, j]
        alpha = np.linalg.norm(x)
        if alpha == 0.0:
            refl.append((j, None))
            continue
        s = 1.0 if x[0] >= 0 else -1.0
        v = x.copy()
        v[0] += s * alpha
        vv = v @ v
        if j + 1 < k:
            w = v @ A[j:, j + 1:]
            A[j:, j + 1:] -= np.multiply.outer(v * (2.0 / vv), w)
        A[j, j] = -s * alpha
        A[j + 1:, j] = 0.0
        refl.append((j, (v, vv)))
    R = np.triu(A[:k, :k])
    sgn = np.ones(k)
    if positive_diag:
        sgn = np.where(np.diag(R) < 0, -1.0, 1.0)
        R = R * sgn[:, None]
    return (refl, sgn), R


def apply_qt(Qinfo, y: np.ndarray) -> np.ndarray:
    """Q^T y (first k entries carry the row signs used for R)."""
    refl, sgn = Qinfo
    z = np.array(y, dtype=np.float64, copy=True)
    for j, rv in refl:
        if rv is None:
            continue
        v, vv = rv
        z[j:] -= v * (2.0 * (v @ z[j:]) / vv)
    z[: len(sgn)] *= sgn
    return z


def back_substitution(R: np.ndarray, y: np.ndarray) -> np.ndarray:
    """Solve R x = y for upper-triangular R, row by row from the bottom."""
    n = R.shape[0]
    x = np.zeros(n)
    for i in range(n - 1, -1, -1):
        x[i] = (y[i] - R[i, i + 1:] @ x[i + 1:]) / R[i, i]
    return x


def forward_substitution_transposed(R: np.ndarray, y: np.ndarray) -> np.ndarray:
    """Solve R^T x = y for upper-triangular R (R^T lower), row by row from the top."""
    n = R.shape[0]
    x = np.zeros(n)
    for i in range(n):
        x[i] = (y[i] - R[:i, i] @ x[:i]) / R[i, i]
    return x


def qr_lstsq(A: np.ndarray, b: np.ndarray) -> np.ndarray:
    """x = argmin ||b - A x|| by Householder QR: R x = (Q^T b)[:n] (eq:ls, classical solver)."""
    m, n = A.shape
    Qinfo, R = householder_qr(A)
    c = apply_qt(Qinfo, b)
    return back_substitution(R, c[:n])


def qr_lstsq_lapack(A: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Same solver with LAPACK's Householder QR (dgeqrf) as the factorization step.

    Used only as the forward-error reference on problems too large for the plain loop above
    (labelled as LAPACK wherever it is reported).
    """
    import scipy.linalg as sl

    Q, R = sl.qr(A, mode="economic")
    return sl.solve_triangular(R, Q.T @ b, lower=False)


# ---------------------------------------------------------------- complex least squares
# The Prony problems of Section 5.2 are complex.  Textbook complex Householder QR: for x = A[k:, k]
# the reflector H = I - 2 v v^H / (v^H v) with v = x + e^{i arg x_0} ||x|| e_1 (e^{i arg 0} = 1)
# maps x to -e^{i arg x_0} ||x|| e_1; H is Hermitian and unitary.  Rows of R are multiplied by a
# unit-modulus phase so that diag(R) is real and non-negative.


def householder_qr_complex(M: np.ndarray):
    """Return ((reflectors, phases), R) for complex M (m x k, m >= k); diag(R) >= 0 real."""
    A = np.array(M, dtype=np.complex128, order="F", copy=True)
    m, k = A.shape
    if m < k:
        raise ValueError("householder_qr_complex expects m >= k")
    refl = []
    for j in range(k):
        x = A[j:, j]
        alpha = np.linalg.norm(x)
        if alpha == 0.0:
            refl.append((j, None))
            continue
        ph = x[0] / abs(x[0]) if x[0] != 0 else 1.0 + 0.0j
        v = x.copy()
        v[0] += ph * alpha
        vv = float(np.real(np.vdot(v, v)))
        if j + 1 < k:
            w = v.conj() @ A[j:, j + 1:]
            A[j:, j + 1:] -= np.multiply.outer(v * (2.0 / vv), w)
        A[j, j] = -ph * alpha
        A[j + 1:, j] = 0.0
        refl.append((j, (v, vv)))
    R = np.triu(A[:k, :k])
    d = np.diag(R)
    rph = np.where(d == 0, 1.0 + 0.0j, d / np.where(d == 0, 1.0, np.abs(d)))
    R = R * rph.conj()[:, None]
    R[np.diag_indices(k)] = np.abs(d)  # exactly real (the product above rounds its imaginary part)
    return (refl, rph), R


def apply_qh_complex(Qinfo, y: np.ndarray) -> np.ndarray:
    """Q^H y for the factorization of householder_qr_complex (first k entries carry the phases)."""
    refl, rph = Qinfo
    z = np.array(y, dtype=np.complex128, copy=True)
    for j, rv in refl:
        if rv is None:
            continue
        v, vv = rv
        z[j:] -= v * (2.0 * np.vdot(v, z[j:]) / vv)
    z[: len(rph)] *= rph.conj()
    return z


def back_substitution_complex(R: np.ndarray, y: np.ndarray) -> np.ndarray:
    n = R.shape[0]
    x = np.zeros(n, dtype=np.complex128)
    for i in range(n - 1, -1, -1):
        x[i] = (y[i] - R[i, i + 1:] @ x[i + 1:]) / R[i, i]
    return x


def qr_lstsq_complex(A: np.ndarray, b: np.ndarray) -> np.ndarray:
    """x = argmin ||b - A x|| over C^n by complex Householder QR: R x = (Q^H b)[:n]."""
    m, n = A.shape
    Qinfo, R = householder_qr_complex(A)
    c = apply_qh_complex(Qinfo, b)
    return back_substitution_complex(R, c[:n])
