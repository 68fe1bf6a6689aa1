"""Generators for the synthetic least-squares test problems (inputs only, no solver arithmetic).

``make_problem`` runs on the CPU with numpy and is bit-reproducible from its seed; it is used for
every size the CPU can build in seconds (up to ~1e5 x 1e3).  ``make_problem_torch`` builds the same
distribution directly in device memory for the 1e6 x 1e3 problems; its random stream is torch's,
so its bytes differ from the numpy generator's for the same seed, and every consumer of such a
problem (oracle-side checks included) reads the bytes it produced.

Recipe (paper, Section 1, description of the Figure 1 problem; Section 5.1 for the sweeps):
  * U = Q factor of an m x n standard Gaussian matrix with the signs of diag(R) made positive
    (the Haar measure on the Stiefel manifold), likewise V (n x n);
  * sigma_i = 10^{p_i}, p_i equally spaced from 0 to -log10(kappa);
  * A = U diag(sigma) V^T, stored column-major (Fortran order);
  * x_true ~ N(0, I_n);
  * r_perp = radius * P g / ||P g||, g ~ N(0, I_m), P = I - U U^T (applied twice);
  * b = A x_true + r_perp.
"""

from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np


@dataclass
class Problem:
    A: "np.ndarray | object"          # m x n, column-major (numpy Fortran order or torch (m,n) with strides (1,m))
    b: "np.ndarray | object"          # m
    x_true: np.ndarray                 # n
    sigma: np.ndarray                  # n, the exact singular values of U diag(sigma) V^T
    V: np.ndarray                      # n x n right singular vectors
    kappa: float
    resid_norm: float
    seed: int
    U: Optional[np.ndarray] = None     # m x n left singular vectors (small problems only)
    meta: dict = field(default_factory=dict)

    @property
    def shape(self):
        return tuple(self.A.shape)


def log_spaced_sigma(n: int, kappa: float) -> np.ndarray:
    """sigma_i = 10^{p_i}, p_i equally spaced in [0, -log10(kappa)] (Figure 1 description)."""
    if n == 1:
        return np.ones(1)
    return 10.0 ** (-np.linspace(0.0, np.log10(kappa), n))


def _positive_diag_qr(G: np.ndarray) -> np.ndarray:
    import scipy.linalg as sl

    Q, R = sl.qr(G, mode="economic")
    s = np.sign(np.diag(R))
    s[s == 0] = 1.0
    return Q * s


def haar_cholqr2(G: np.ndarray) -> np.ndarray:
    """Orthonormal Q of the positive-diagonal QR of a well-conditioned Gaussian G (m >= 4n).

    Two rounds of Cholesky QR; the product of the two Cholesky factors has a positive diagonal, so
    Q is the same Q as Householder QR with the sign fix, up to rounding.
    """
    import scipy.linalg as sl

    Q = np.asfortranarray(G)
    for _ in range(2):
        C = Q.T @ Q
        L = np.linalg.cholesky(C)                      # C = L L^T, R = L^T
        Q = sl.solve_triangular(L, Q.T, lower=True).T  # Q R^{-1}
    return np.asfortranarray(Q)


def _haar(rng: np.random.Generator, m: int, n: int) -> np.ndarray:
    G = rng.standard_normal((m, n))
    if m >= 4 * n:
        return haar_cholqr2(G)
    return _positive_diag_qr(G)


def make_problem(m: int, n: int, kappa: float, resid_norm: float, seed: int,
                 keep_U: Optional[bool] = None) -> Problem:
    """CPU (numpy) generator; deterministic from ``seed``."""
    if not (m >= n >= 1):
        raise ValueError("need m >= n >= 1")
    rng = np.random.default_rng(seed)
    U = _haar(rng, m, n)
    V = _haar(rng, n, n)
    sigma = log_spaced_sigma(n, kappa)
    A = np.asfortranarray((U * sigma) @ V.T)
    x_true = rng.standard_normal(n)
    g = rng.standard_normal(m)
    r = g - U @ (U.T @ g)
    r = r - U @ (U.T @ r)
    nr = np.linalg.norm(r)
    r = r * (resid_norm / nr) if nr > 0 else r
    b = A @ x_true + r
    if keep_U is None:
        keep_U = m * n <= 4_000_000
    return Problem(A=A, b=b, x_true=x_true, sigma=sigma, V=V, kappa=float(kappa),
                   resid_norm=float(resid_norm), seed=int(seed), U=U if keep_U else None,
                   meta={"generator": "numpy", "r_perp": r if keep_U else None})


def make_multi_problem(m: int, n: int, kappa: float, resid_norms, k: int, seed: int) -> Problem:
    """CPU generator with k right-hand sides sharing A (same recipe as ``make_problem``):
    column j of B is A x_j + r_j with x_j ~ N(0, I_n) and r_j perpendicular to range(A), of norm
    resid_norms[j % len(resid_norms)] (0 gives b_j = A x_j exactly in exact arithmetic).
    ``meta["B"]`` (m x k, Fortran order) and ``meta["X_true"]`` (n x k) hold them."""
    rng = np.random.default_rng(seed)
    U = _haar(rng, m, n)
    V = _haar(rng, n, n)
    sigma = log_spaced_sigma(n, kappa)
    A = np.asfortranarray((U * sigma) @ V.T)
    norms = list(resid_norms)
    Xt = rng.standard_normal((n, k))
    G = rng.standard_normal((m, k))
    Rp = G - U @ (U.T @ G)
    Rp = Rp - U @ (U.T @ Rp)
    for j in range(k):
        nr = np.linalg.norm(Rp[:, j])
        Rp[:, j] *= norms[j % len(norms)] / nr if nr > 0 else 0.0
    B = np.asfortranarray(A @ Xt + Rp)
    return Problem(A=A, b=B[:, 0].copy(), x_true=Xt[:, 0].copy(), sigma=sigma, V=V, kappa=float(kappa),
                   resid_norm=float(norms[0]), seed=int(seed), U=U if m * n <= 4_000_000 else None,
                   meta={"generator": "numpy", "B": B, "X_true": Xt, "rhs_resid_norms": norms})


def make_problem_torch(m: int, n: int, kappa: float, resid_norm: float, seed: int,
                       device: str = "cuda", nrhs: int = 0, rhs_resid_norms=None) -> Problem:
    """Device-side generator for the large (1e6 x 1e3) problems.

    V, sigma and x_true come from numpy (small); U, A and b are formed in device memory with
    torch's seeded generator.  ``A`` is returned as a torch (m, n) float64 tensor with
    column-major strides (1, m).  With ``nrhs > 0`` a column-major (m, nrhs) block ``B`` of
    right-hand sides is also built, column j using solution ``X_true[:, j] ~ N(0, I)`` and residual
    norm ``rhs_resid_norms[j % len(rhs_resid_norms)]``; it is stored in ``meta``.
    """
    import torch

    if not (m >= 4 * n):
        raise ValueError("device generator expects m >= 4n")
    rng = np.random.default_rng(seed)
    V = _haar(rng, n, n)
    sigma = log_spaced_sigma(n, kappa)
    x_true = rng.standard_normal(n)
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed) * 1000003 + 17)
    # U as an (n, m) row-major tensor == (m, n) column-major.
    Ut = torch.randn((n, m), generator=gen, dtype=torch.float64, device=device)
    for _ in range(2):
        C = Ut @ Ut.T                                   # n x n Gram
        L = torch.linalg.cholesky(C)                    # C = L L^T
        Linv = torch.linalg.inv(L)                      # n x n, well conditioned (C ~ m I)
        Ut = Linv @ Ut                                  # L^{-1} U^T = (U L^{-T})^T
    Vt = torch.as_tensor(V, device=device)
    sig = torch.as_tensor(sigma, device=device)
    # A^T = V diag(sigma) U^T  (n x m row-major == A column-major)
    At = (Vt * sig) @ Ut
    xt = torch.as_tensor(x_true, device=device)

    def perp(radius):
        g = torch.randn((m,), generator=gen, dtype=torch.float64, device=device)
        r = g - Ut.T @ (Ut @ g)
        r = r - Ut.T @ (Ut @ r)
        return r * (radius / torch.linalg.norm(r))

    r = perp(resid_norm)
    b = At.T @ xt + r
    meta = {"generator": "torch", "device": device}
    if nrhs > 0:
        norms = list(rhs_resid_norms or [resid_norm])
        Xt = rng.standard_normal((n, nrhs))
        Bt = torch.empty((nrhs, m), dtype=torch.float64, device=device)  # (m, nrhs) column-major
        X_dev = torch.as_tensor(Xt, device=device)
        AX = (At.T @ X_dev)  # m x nrhs
        for j in range(nrhs):
            Bt[j] = AX[:, j] + perp(norms[j % len(norms)])
        meta.update({"B": Bt.T, "X_true": Xt, "rhs_resid_norms": norms})
        del AX
    del Ut
    A = At.T  # (m, n) view with strides (1, m)
    return Problem(A=A, b=b, x_true=x_true, sigma=sigma, V=V, kappa=float(kappa),
                   resid_norm=float(resid_norm), seed=int(seed), U=None, meta=meta)


# ---------------------------------------------------------------- complex-valued problems
#
# Section 5.2's second dense workload is complex (Prony's method, Appendix B).  Two generators:
#   * make_complex_problem: the Figure 1 recipe over C (complex Haar U, V from the QR of complex
#     Gaussian matrices with a positive real diag(R); A = U diag(sigma) V^H; x_true and r_perp
#     complex Gaussian, r_perp in the orthogonal complement of range(A));
#   * make_prony_problem: the first least-squares solve of Prony's method (Appendix B, line 1 of
#     its algorithm): samples f_j = sum_k mu_k z_k^j + eps_j, j = 0 .. m+n-1, the Toeplitz
#     A = (f_{n-1+i-j}) (1 <= i <= m, 1 <= j <= n) and b = (f_{n-1+i}).  The paper's samples come
#     from a 16-site transverse-field Ising model on a quantum device; here they are synthesized
#     with the same structure: K unit-modulus z_k = exp(-i dt lambda_k) for eigenvalues lambda_k
#     drawn uniformly in [-1, 1], positive weights mu_k decaying like exp(-3 k / K) (a few
#     dominant overlaps, normalized to sum 1) and complex Gaussian noise eps_j of standard
#     deviation `noise` (1e-6 in the paper).  With K < n the noise-free system is consistent and
#     rank deficient, so the noise sets condition number and residual: K = 10, n = 100,
#     m = 20000 gives about 4e6 and 2e-6 (the paper reports about 1e6 and 1e-6).


@dataclass
class ComplexProblem:
    A: np.ndarray                      # m x n complex128, column-major
    b: np.ndarray                      # m complex128
    x_true: Optional[np.ndarray]       # n (None for Prony problems)
    sigma: Optional[np.ndarray]        # exact singular values when known
    V: Optional[np.ndarray]            # n x n right singular vectors when known
    kappa: float
    meta: dict = field(default_factory=dict)


def _complex_haar(rng: np.random.Generator, m: int, n: int) -> np.ndarray:
    import scipy.linalg as sl

    G = rng.standard_normal((m, n)) + 1j * rng.standard_normal((m, n))
    Q, R = sl.qr(G, mode="economic")
    d = np.diag(R)
    ph = np.where(d == 0, 1.0, d / np.abs(d))
    return np.asfortranarray(Q * ph)


def make_complex_problem(m: int, n: int, kappa: float, resid_norm: float, seed: int) -> ComplexProblem:
    if not (m >= n >= 1):
        raise ValueError("need m >= n >= 1")
    rng = np.random.default_rng(seed)
    U = _complex_haar(rng, m, n)
    V = _complex_haar(rng, n, n)
    sigma = log_spaced_sigma(n, kappa)
    A = np.asfortranarray((U * sigma) @ V.conj().T)
    x_true = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    g = rng.standard_normal(m) + 1j * rng.standard_normal(m)
    r = g - U @ (U.conj().T @ g)
    r = r - U @ (U.conj().T @ r)
    nr = np.linalg.norm(r)
    r = r * (resid_norm / nr) if nr > 0 else r
    b = A @ x_true + r
    return ComplexProblem(A=A, b=b, x_true=x_true, sigma=sigma, V=V, kappa=float(kappa),
                          meta={"resid_norm": float(resid_norm), "seed": int(seed), "U": U if m * n <= 4_000_000 else None})


def prony_samples(count: int, K: int, noise: float, seed: int, dt: float = 1.0):
    """f_j = sum_k mu_k z_k^j + eps_j for j < count; returns (f, z, mu)."""
    rng = np.random.default_rng(seed)
    lam = np.sort(rng.uniform(-1.0, 1.0, K))
    z = np.exp(-1j * dt * lam)
    mu = np.exp(-3.0 * np.arange(K) / K) * rng.uniform(0.5, 1.0, K)  # a few dominant overlaps
    mu = mu / mu.sum()
    j = np.arange(count)
    f = np.zeros(count, dtype=np.complex128)
    for k in range(K):  # z_k^j through the angle (exact unit modulus for every j)
        f += mu[k] * np.exp(-1j * dt * lam[k] * j)
    f += noise * (rng.standard_normal(count) + 1j * rng.standard_normal(count)) / np.sqrt(2.0)
    return f, z, mu


def make_prony_problem(m: int, n: int, K: int, noise: float = 1e-6, seed: int = 0, dt: float = 1.0) -> ComplexProblem:
    if not (m >= n >= 1) or K < 1:
        raise ValueError("need m >= n >= 1 and K >= 1")
    f, z, mu = prony_samples(m + n, K, noise, seed, dt)
    i = np.arange(1, m + 1)[:, None]
    jj = np.arange(1, n + 1)[None, :]
    A = np.asfortranarray(f[n - 1 + i - jj])
    b = f[n - 1 + np.arange(1, m + 1)].copy()
    return ComplexProblem(A=A, b=b, x_true=None, sigma=None, V=None, kappa=float("nan"),
                          meta={"z": z, "mu": mu, "K": K, "noise": noise, "seed": seed, "dt": dt})
