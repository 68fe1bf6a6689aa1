"""Sparse sign embedding S and the sketch S [A b] -- oracle side (test infrastructure only).

Paper, Section 4.2 ("Choice of embedding"): S = zeta^{-1/2} [s_1 ... s_m] is d x m; column s_j has
zeta nonzeros +-1 at uniformly random distinct positions (the paper writes s_i in R^m, read here as
R^d since S has d rows).  Algorithm 1 sketches [A b] together so that the QR of the sketch also
yields Q^T (S b).

The product is formed as plain signed sums in float64 in increasing source row j (scipy's CSR
product walks each row of S in increasing column order), followed by one multiplication by
fl(1/sqrt(zeta)).
"""

from __future__ import annotations

import numpy as np

from .philox import sparse_sign_indices


def sparse_sign_matrix(m: int, d: int, zeta: int, seed: int):
    """S without its zeta^{-1/2} factor, as a scipy CSR matrix (d x m) of +-1 entries."""
    import scipy.sparse as sp

    rows, signs = sparse_sign_indices(m, d, zeta, seed)
    cols = np.repeat(np.arange(m, dtype=np.int64), zeta)
    S = sp.coo_matrix((signs.reshape(-1).astype(np.float64), (rows.reshape(-1).astype(np.int64), cols)),
                      shape=(d, m)).tocsr()
    S.sort_indices()
    return S


def dense_sign_matrix(m: int, d: int, zeta: int, seed: int) -> np.ndarray:
    """Dense S including the zeta^{-1/2} factor; for tiny m only (reference for the sparse path)."""
    rows, signs = sparse_sign_indices(m, d, zeta, seed)
    S = np.zeros((d, m))
    for j in range(m):
        for k in range(zeta):
            S[rows[j, k], j] = signs[j, k]
    return S / np.sqrt(zeta)


def sketch(M: np.ndarray, d: int, zeta: int, seed: int) -> np.ndarray:
    """S M for an m x k matrix M (or an m-vector); returns d x k (Fortran order)."""
    M2 = M.reshape(M.shape[0], -1)
    S = sparse_sign_matrix(M2.shape[0], d, zeta, seed)
    Y = np.asfortranarray(S @ M2)
    Y *= 1.0 / np.sqrt(zeta)
    return Y if M.ndim == 2 else Y[:, 0]


def sketch_Ab(A: np.ndarray, b: np.ndarray, d: int, zeta: int, seed: int) -> np.ndarray:
    """Y = S [A b], d x (n+1) (Algorithm 1, first statement: one embedding for [A b])."""
    return sketch(np.column_stack([A, b]), d, zeta, seed)


def sketch_fp32(M: np.ndarray, d: int, zeta: int, seed: int) -> np.ndarray:
    """The mixed-precision form's sketch: S fl32(M), the sketch of the single-precision copy, with
    double-precision sums.  Each entry is within (u32 + (k + 2) u) (|S| |M|) of S M, k the entry's
    count of nonzero terms."""
    M32 = np.asarray(M, dtype=np.float32).astype(np.float64)
    return sketch(M32, d, zeta, seed)
