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


def _tsqr_r(M_of_rows, m: int, k: int, block_rows: int, workers: int) -> np.ndarray:
    """Triangular factor (k x k) of an m x k matrix given by row blocks, by TSQR: LAPACK's
    Householder QR (dgeqrf) of each block of rows, then the same on the stacked triangles until
    one block remains."""
    import scipy.linalg as sl
    from concurrent.futures import ThreadPoolExecutor

    from threadpoolctl import threadpool_limits

    def leaf(i0, i1):
        M = np.array(M_of_rows(i0, i1), dtype=np.float64, order="F", copy=True)
        R = sl.qr(M, mode="r", overwrite_a=True, check_finite=False)[0]
        return R[: min(k, i1 - i0)]

    bounds = [(i, min(m, i + block_rows)) for i in range(0, m, block_rows)]
    # one LAPACK thread per block, the blocks spread over the workers
    with threadpool_limits(1), ThreadPoolExecutor(max(1, workers)) as ex:
        Rs = list(ex.map(lambda bl: leaf(*bl), bounds))
    while len(Rs) > 1:
        stacked = np.vstack(Rs)
        group = max(2, block_rows // k)
        parts = [stacked[i:i + group * k] for i in range(0, stacked.shape[0], group * k)]
        if len(parts) == 1:
            Rs = [sl.qr(np.asfortranarray(parts[0]), mode="r", check_finite=False)[0][:k]]
            break
        with threadpool_limits(1), ThreadPoolExecutor(max(1, workers)) as ex:
            Rs = list(ex.map(lambda p: sl.qr(np.asfortranarray(p), mode="r", check_finite=False)[0][:k], parts))
    R = Rs[0]
    if R.shape[0] < k:
        R = np.vstack([R, np.zeros((k - R.shape[0], k))])
    return np.triu(R)


def qr_lstsq_tsqr(A: np.ndarray, B: np.ndarray, block_rows: int = 5000, workers: int = 0) -> np.ndarray:
    """Householder-QR least squares for a tall A (m x n) and one or more right-hand sides B (m or
    m x k), as the forward-error reference at sizes where the plain loop above is out of reach.

    The augmented matrix [A B] is reduced to triangular form by TSQR (Demmel, Grigori, Hoemmen,
    Langou, "Communication-optimal parallel and sequential QR and LU factorizations", 2012):
    LAPACK's Householder QR of row blocks, then of the stacked triangles.  The result is the
    triangle of a Householder QR of [A B] = Q [R T; 0 *], whose leading columns give R and T =
    (Q^T B)[:n]; x = R^{-1} T.  A sequence of Householder reflections, so the solver keeps the
    backward stability of Householder QR least squares (labelled "LAPACK TSQR" where reported).
    """
    import os

    import scipy.linalg as sl

    A = np.asarray(A)
    Bm = np.asarray(B, dtype=np.float64)
    vec = Bm.ndim == 1
    if vec:
        Bm = Bm[:, None]
    m, n = A.shape
    k = Bm.shape[1]
    if m < n:
        raise ValueError("qr_lstsq_tsqr expects m >= n")
    workers = workers or min(16, os.cpu_count() or 1)
    block_rows = max(block_rows, 2 * (n + k))

    def rows(i0, i1):
        M = np.empty((i1 - i0, n + k), order="F")
        M[:, :n] = A[i0:i1]
        M[:, n:] = Bm[i0:i1]
        return M

    Rt = _tsqr_r(rows, m, n + k, block_rows, workers)
    X = sl.solve_triangular(Rt[:n, :n], Rt[:n, n:], lower=False, check_finite=False)
    return X[:, 0] if vec else X


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
