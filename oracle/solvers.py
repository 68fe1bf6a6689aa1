"""FOSSILS and SPIR -- oracle side (test infrastructure only).

Written from the paper's algorithms in their order and notation:
  * Algorithm 1 (meta-algorithm): sketch [A b], QR of S A, sketch-and-solve x_0
    (eq:sketch-and-solve-2.3), then exactly two refinement steps
    c_i = P^T A^T (b - A x_i),  dy_i = IterativeSolver(z -> P^T A^T A P z, c_i),
    x_{i+1} = x_i + P dy_i  (eq:precond-normal-RHSc).
  * Algorithm 5 (Polyak heavy ball) with eq:optimal-coeffs alpha = (1 - eta^2)^2, beta = eta^2;
    Algorithm 2 runs it a fixed q times, Theorem 7.1 (eq:iterations) gives q_0.
  * Algorithm 4 (recommended FOSSILS): column scaling, d = 12 n, zeta = 8, SVD of the sketch,
    rank truncation at tau = 30 u, P = V Sigma^{-1}, and the two adaptive stopping rules of
    Section 4.2 ("Adaptive stopping"), with these readings of garbled statements:
      - "beta <- d/n" is read as beta = eta^2 = n/d (eq:optimal-coeffs, Algorithm 2);
      - the "+ mu^2 z" term is dropped (mu = 0; the paper implements truncation instead of
        regularization);
      - the "Mod(i, 5)" test of the second step is read on the inner index j;
      - the first-step rule uses ||x_0|| and ||b - A x_0|| (Section 4.2's statement).
  * SPIR (Algorithm 3) with conjugate gradient on the preconditioned normal equations and the
    same stopping rules (the paper omits its practical version; Delta = a_k p_k).
  * Unit roundoff u = 2^-52.

Preconditioner choices: ``precond="svd"`` is Algorithm 4's P = V Sigma^{-1} from the SVD of S A;
``precond="qr"`` is Algorithms 1-3's P = R^{-1} from Householder QR of S [A b], applied by back
substitution (Section 6: triangular solves are back substitutions); Sigma and V for the
stopping rules then come from the SVD of R (S A = (Q U_R) Sigma V^T).  A numerically
rank-deficient sketch always falls back to the truncated SVD preconditioner (Alg 4).
"""

from __future__ import annotations

import math
import time
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

from .backward_error import kw_from_svd
from .householder import back_substitution, forward_substitution_transposed, householder_qr
from .sketch import sketch_Ab, sketch_fp32

U_ROUND = 2.0**-52

FLAG_RANK_DEFICIENT = 1
FLAG_NOT_CONVERGED = 2
FLAG_FP64_SKETCH = 4

U32 = 2.0**-24
# mixed precision: the sketch of the FP32 copy is kept while u32 condest <= 2 (see solve()); measured
# with this oracle on 4000 x 50 problems (fallback disabled), that preconditioner needs the FP64
# iteration counts up to u32 condest ~ 6 (kappa = 1e8), three times as many at ~ 10 and fails to
# converge beyond ~ 11 (kappa >= 1e9)
MIXED_COND_FACTOR = U32
MIXED_DISTORTION = 2.0


@dataclass
class Options:
    d: Optional[int] = None          # sketch rows; default 12 n (Alg 4)
    zeta: int = 8                    # nonzeros per column of S (Alg 4)
    seed: int = 12345                # sketch seed
    eta: Optional[float] = None      # distortion estimate; default sqrt(n/d) (Section 4.2)
    eta_factor: float = 1.0          # 1.1 = the paper's conservative choice
    gamma: float = 10.0              # first-step rule constants of Alg 4
    rho: float = 0.4
    kw_every: int = 5                # sketched-KW cadence in the second step
    max_inner: int = 100             # iteration cap per refinement step (Alg 4)
    tau_factor: float = 30.0         # truncation threshold tau = 30 u
    column_scaling: bool = True
    precond: str = "qr"              # "qr" (P = R^{-1}) or "svd" (P = V Sigma^{-1})
    fixed_q: int = 0                 # 0 adaptive; q > 0 Algorithm 2 with q steps; -1 q_0 of Thm 7.1
    steps: int = 2                   # refinement steps (2 = the method; 1 = "FOSSILS (1 step)")
    precision: str = "fp64"          # "fp64", or "mixed": FP32 sketch, FP64 everything else
    init: str = "sketch"             # "sketch": x_0 = sketch-and-solve (Alg 4); "zero": x_0 = 0
    mixed_fallback: bool = True      # mixed: redo the sketch in FP64 when condest u32 is too large


@dataclass
class Result:
    x: np.ndarray
    iters: list
    flags: int
    normest: float
    condest: float
    rank: int
    be_sk: float
    x0: np.ndarray
    xs: list = field(default_factory=list)     # iterate after each refinement step (unscaled)
    cs: list = field(default_factory=list)     # ||c_i|| (Table 2 quantity)
    info: dict = field(default_factory=dict)


# ---------------------------------------------------------------- single passes over A

def column_norms(A):
    """d_j = ||a_j||_2 (Alg 4, first statement); zero columns get 1 so the scaling is defined."""
    d = np.sqrt(np.sum(A * A, axis=0))
    d[d == 0.0] = 1.0
    return d


def normal_pass(A, z):
    """v = A^T (A z): the operator of the preconditioned normal equations (eq:precond-normal)."""
    return A.T @ (A @ z)


def residual_pass(A, b, x):
    """r = b - A x, g = A^T r and ||r||^2 (Algorithm 1, the refinement right-hand side)."""
    r = b - A @ x
    return A.T @ r, float(r @ r)


def polyak(apply_M, c, alpha, beta, q):
    """Algorithm 5: dy_(1) = dy_(0) = c, then q - 1 heavy-ball updates
    dy_(j+1) = dy_(j) + alpha (c - M dy_(j)) + beta (dy_(j) - dy_(j-1))."""
    dy = c.copy()
    dy_old = c.copy()
    for _ in range(1, q):
        dy, dy_old = dy + alpha * (c - apply_M(dy)) + beta * (dy - dy_old), dy
    return dy


def polyak_coefficients(eta):
    """eq:optimal-coeffs: alpha = (1 - eta^2)^2, beta = eta^2."""
    beta = eta * eta
    return (1.0 - beta) ** 2, beta


def lsqr_iterate(apply_B, apply_BT, r, c, q):
    """Paige and Saunders' LSQR for min || r - B y || from y = 0, given c = B^T r: Golub-Kahan
    bidiagonalization (beta_1 u_1 = r, alpha_1 v_1 = B^T u_1 = c / beta_1, then
    beta u' = B v - alpha u, alpha v' = B^T u' - beta v) with a Givens rotation per step.  Yields
    (Delta, y, done) after each of at most q steps; Delta is the step's update of y, done is set when
    the bidiagonalization terminates (alpha or beta = 0: y is the exact minimizer)."""
    bet = float(np.linalg.norm(r))
    cn = float(np.linalg.norm(c))
    y = np.zeros_like(c)
    if bet == 0.0 or cn == 0.0:
        return
    uvec = r / bet
    alf = cn / bet
    vvec = c / cn
    w = vvec.copy()
    phibar, rhobar = bet, alf
    for _ in range(q):
        t = apply_B(vvec) - alf * uvec
        bet = float(np.linalg.norm(t))
        if bet > 0.0:
            uvec = t / bet
        s_v = apply_BT(uvec) - bet * vvec
        alf = float(np.linalg.norm(s_v))
        if alf > 0.0:
            vvec = s_v / alf
        rho = math.hypot(rhobar, bet)
        cs, sn = rhobar / rho, bet / rho
        theta = sn * alf
        rhobar = -cs * alf
        phi = cs * phibar
        phibar = sn * phibar
        Delta = (phi / rho) * w
        y = y + Delta
        w = vvec - (theta / rho) * w
        yield Delta, y, (bet == 0.0 or alf == 0.0)


def q0_theorem71(kappa, eta):
    """eq:iterations: q_0 = max(1 + 2 log(1/(kappa u)) / log(1/(1.01 eta)), 11), rounded up."""
    ku = kappa * U_ROUND
    if ku >= 1.0:
        return 11
    return int(math.ceil(max(1.0 + 2.0 * math.log(1.0 / ku) / math.log(1.0 / (1.01 * eta)), 11.0)))


# ---------------------------------------------------------------- the solver

class _Precond:
    """P and P^T for either preconditioner (R^{-1} by substitution, or V Sigma^{-1})."""

    def __init__(self, kind, R=None, V=None, sigma=None):
        self.kind, self.R, self.V, self.sigma = kind, R, V, sigma

    def P(self, y):
        if self.kind == "qr":
            return back_substitution(self.R, y)
        return self.V @ (y / self.sigma)

    def PT(self, v):
        if self.kind == "qr":
            return forward_substitution_transposed(self.R, v)
        return (self.V.T @ v) / self.sigma


def _stop_first(Delta, thr):
    return np.linalg.norm(Delta) <= thr


def solve(A, b, method="fossils", opts: Optional[Options] = None) -> Result:
    """FOSSILS (Algorithm 4 / Algorithm 2), SPIR (Algorithm 3 with CG) or SPIR with LSQR
    (method "spir_lsqr") for min ||b - A x||."""
    opts = opts or Options()
    A = np.asarray(A, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    m, n = A.shape
    if not (m >= n >= 1):
        raise ValueError("need m >= n >= 1")
    if not (np.all(np.isfinite(A)) and np.all(np.isfinite(b))):
        raise ValueError("non-finite input")
    dsk = opts.d or 12 * n
    if dsk < n or not (1 <= opts.zeta <= dsk):
        raise ValueError("need n <= d and 1 <= zeta <= d")
    u = U_ROUND
    if np.linalg.norm(b) == 0.0:
        z = np.zeros(n)
        return Result(x=z, iters=[0, 0], flags=0, normest=0.0, condest=0.0, rank=n, be_sk=0.0, x0=z)

    # Wall-clock marks of the phases (reported in info["phase_s"]; no effect on the arithmetic).
    marks = [("start", time.perf_counter())]
    # Alg 4: normalize columns.
    dcol = column_norms(A) if opts.column_scaling else np.ones(n)
    As = A / dcol
    # Alg 4: embedding parameters and Polyak coefficients.
    eta = (opts.eta if opts.eta is not None else math.sqrt(n / dsk)) * opts.eta_factor
    alpha, beta = polyak_coefficients(eta)
    # Alg 1 / Alg 4: sketch [A b] with one embedding (of the single-precision copy of A in the mixed
    # form, whose column norms then give the scaling).
    flags = 0
    if opts.precision == "mixed":
        A32 = A.astype(np.float32).astype(np.float64)
        dcol32 = column_norms(A32) if opts.column_scaling else np.ones(n)
        Y = sketch_Ab(A32 / dcol32, b, dsk, opts.zeta, opts.seed)
        # The sketch of fl32(A) is S A perturbed by ~u32 ||A||: R from it preconditions A_s well only
        # while condest u32 is small (Lemma 6.3 with u32 in place of u); beyond that, redo it in FP64.
        cond32 = np.linalg.cond(np.linalg.qr(Y[:, :n], mode="r"))
        if opts.mixed_fallback and not (cond32 * MIXED_COND_FACTOR <= MIXED_DISTORTION):
            flags |= FLAG_FP64_SKETCH
            Y = sketch_Ab(As, b, dsk, opts.zeta, opts.seed)
        else:
            dcol = dcol32
            As = A / dcol
    elif opts.precision == "fp64":
        Y = sketch_Ab(As, b, dsk, opts.zeta, opts.seed)
    else:
        raise ValueError("precision must be 'fp64' or 'mixed'")
    SA, Sb = Y[:, :n], Y[:, n]
    marks.append(("sketch", time.perf_counter()))

    # Factor the sketch.
    if opts.precond == "qr":
        Qinfo, Rfull = householder_qr(Y)          # S[A b] = Q [R t; 0 rho]
        R, t = Rfull[:n, :n], Rfull[:n, n]
        _, sig_full, Vt = np.linalg.svd(R)         # S A = (Q U_R) Sigma V^T
        V_full = Vt.T
        U_R = None
    elif opts.precond == "svd":
        U_sk, sig_full, Vt = np.linalg.svd(SA, full_matrices=False)
        V_full = Vt.T
        R = t = None
    else:
        raise ValueError("precond must be 'qr' or 'svd'")
    marks.append(("factor", time.perf_counter()))
    normest = float(sig_full[0])
    condest = float(sig_full[0] / sig_full[-1]) if sig_full[-1] > 0 else math.inf

    rank = n
    kind = opts.precond
    if condest > 1.0 / (opts.tau_factor * u):
        # Alg 4: numerically rank deficient -> truncated SVD preconditioner.
        flags |= FLAG_RANK_DEFICIENT
        rank = int(np.sum(sig_full > opts.tau_factor * u * normest))
        kind = "svd"
        if opts.precond == "qr":
            U_R, _, _ = np.linalg.svd(R)
    if kind == "svd":
        sig = sig_full[:rank]
        V = V_full[:, :rank]
        pre = _Precond("svd", V=V, sigma=sig)
        if opts.precond == "svd":
            x0 = V @ ((U_sk[:, :rank].T @ Sb) / sig)          # Alg 4 sketch-and-solve
        else:
            x0 = V @ ((U_R[:, :rank].T @ t) / sig)            # same with S A = (Q U_R) Sigma V^T
    else:
        pre = _Precond("qr", R=R)
        x0 = back_substitution(R, t)                           # eq:sketch-and-solve-2.3

    if opts.init == "zero":      # sketch-and-precondition's zero start (Section 5.1 comparison)
        x0 = np.zeros(n)
    elif opts.init != "sketch":
        raise ValueError("init must be 'sketch' or 'zero'")
    # Alg 4: r = b - A x, kept for the first-step rule.
    r0 = b - As @ x0
    thr_first = (opts.gamma * normest * np.linalg.norm(x0) + opts.rho * condest * np.linalg.norm(r0)) * u
    fro = np.linalg.norm(As)
    theta = fro / np.linalg.norm(b)

    if opts.fixed_q != 0:
        if opts.fixed_q < 0:
            q = q0_theorem71(condest, eta)
            alpha, beta = polyak_coefficients(1.01 * eta)      # Thm 7.1 (D)
        else:
            q = opts.fixed_q

    def apply_M(y):
        return pre.PT(As.T @ (As @ pre.P(y)))

    marks.append(("x0", time.perf_counter()))
    x = x0.copy()
    iters, xs, cs = [], [], []
    be_sk = math.nan
    converged_last = False
    for i in range(opts.steps):
        c = pre.PT(As.T @ (b - As @ x))
        cs.append(float(np.linalg.norm(c)))
        it = 0
        converged = False
        if method == "fossils" and opts.fixed_q != 0:
            dy = polyak(apply_M, c, alpha, beta, q)               # Algorithm 5
            it = q - 1
            converged = True
        elif method == "fossils":
            dy = c.copy()
            dy_old = c.copy()
            for j in range(opts.max_inner):
                Delta = alpha * (c - apply_M(dy)) + beta * (dy - dy_old)
                dy, dy_old = dy + Delta, dy
                it += 1
                if i == 0 and _stop_first(Delta, thr_first):
                    converged = True
                    break
                if i == 1 and j % opts.kw_every == 0:
                    xh = x + pre.P(dy)
                    rh = b - As @ xh
                    be_sk = kw_from_svd(sig_full, V_full, As.T @ rh, theta, np.linalg.norm(rh), np.linalg.norm(xh))
                    if be_sk < fro * u:
                        converged = True
                        break
        elif method == "spir":
            dy = np.zeros_like(c)
            res = c.copy()
            p = c.copy()
            rho = float(res @ res)
            for j in range(opts.max_inner):
                if rho == 0.0:
                    converged = True
                    break
                qv = apply_M(p)
                pq = float(p @ qv)
                if pq <= 0.0:
                    break
                a = rho / pq
                Delta = a * p
                dy = dy + Delta
                res = res - a * qv
                rho_new = float(res @ res)
                p = res + (rho_new / rho) * p
                rho = rho_new
                it += 1
                if i == 0 and _stop_first(Delta, thr_first):
                    converged = True
                    break
                if i == 1 and j % opts.kw_every == 0:
                    xh = x + pre.P(dy)
                    rh = b - As @ xh
                    be_sk = kw_from_svd(sig_full, V_full, As.T @ rh, theta, np.linalg.norm(rh), np.linalg.norm(xh))
                    if be_sk < fro * u:
                        converged = True
                        break
        elif method == "spir_lsqr":
            # LSQR on min || r_i - (A_s P) dy || (the LSQR form of SPIR, Section 4.3); the stopping
            # rules are SPIR's with Delta = the update of dy.
            dy = np.zeros_like(c)
            steps = lsqr_iterate(lambda y: As @ pre.P(y), lambda v: pre.PT(As.T @ v), b - As @ x, c,
                                 opts.max_inner)
            for j, (Delta, dy, done) in enumerate(steps):
                it += 1
                if done:
                    converged = True
                    break
                if i == 0 and _stop_first(Delta, thr_first):
                    converged = True
                    break
                if i == 1 and j % opts.kw_every == 0:
                    xh = x + pre.P(dy)
                    rh = b - As @ xh
                    be_sk = kw_from_svd(sig_full, V_full, As.T @ rh, theta, np.linalg.norm(rh), np.linalg.norm(xh))
                    if be_sk < fro * u:
                        converged = True
                        break
            else:
                converged = converged or it == 0
        else:
            raise ValueError("method must be 'fossils', 'spir' or 'spir_lsqr'")
        x = x + pre.P(dy)                                     # Alg 1: x_{i+1} = x_i + P dy_i
        iters.append(it)
        xs.append(x / dcol)
        converged_last = converged
        marks.append((f"step{i}", time.perf_counter()))
    if opts.steps == 2 and opts.fixed_q == 0 and not converged_last:
        flags |= FLAG_NOT_CONVERGED
    return Result(x=x / dcol, iters=iters, flags=flags, normest=normest, condest=condest, rank=rank,
                  be_sk=float(be_sk), x0=x0 / dcol, xs=xs, cs=cs,
                  info={"alpha": alpha, "beta": beta, "eta": eta, "d": dsk, "theta": theta,
                        "fro": fro, "dcol": dcol, "thr_first": thr_first,
                        "phase_s": {marks[k][0]: marks[k][1] - marks[k - 1][1] for k in range(1, len(marks))}})


def fossils(A, b, opts: Optional[Options] = None) -> Result:
    return solve(A, b, "fossils", opts)


def fossils_multi(A, B, opts: Optional[Options] = None):
    """Several right-hand sides sharing A: column j of B solved by Algorithm 4 on its own, with the
    same embedding S for every column (the multi-RHS form sketches [A B] with one S, so each
    column sees exactly the sketch [S A, S b_j] of the single-column method).  Returns the list of
    per-column Results."""
    B = np.asarray(B)
    return [fossils(A, B[:, j], opts) for j in range(B.shape[1])]


def spir(A, b, opts: Optional[Options] = None) -> Result:
    return solve(A, b, "spir", opts)


def spir_lsqr(A, b, opts: Optional[Options] = None) -> Result:
    """SPIR with LSQR as the Krylov method of each refinement step (Section 4.3)."""
    return solve(A, b, "spir_lsqr", opts)


def sketch_and_solve(A, b, d, zeta=8, seed=12345):
    """x_0 = R^{-1} (Q^T S b) from the QR of S [A b] (eq:sketch-and-solve-2.3), unscaled A."""
    n = A.shape[1]
    Y = sketch_Ab(A, b, d, zeta, seed)
    _, Rfull = householder_qr(Y)
    return back_substitution(Rfull[:n, :n], Rfull[:n, n])


# ---------------------------------------------------------------- complex problems (Section 5.2)

def realify(A, b):
    """A_R = [Re A, -Im A; Im A, Re A], b_R = [Re b; Im b]: ||A_R [Re x; Im x] - b_R|| = ||A x - b||."""
    Ar = np.block([[A.real, -A.imag], [A.imag, A.real]])
    return np.asfortranarray(Ar), np.concatenate([b.real, b.imag])


def solve_complex(A, b, method="fossils", opts: Optional[Options] = None) -> Result:
    """FOSSILS / SPIR for complex A, b: the real method on the realification, x = x_R[:n] + i x_R[n:]
    (the sketch has 12 (2n) rows by default)."""
    n = A.shape[1]
    Ar, br = realify(A, b)
    res = solve(Ar, br, method, opts)
    res.x = res.x[:n] + 1j * res.x[n:]
    res.x0 = res.x0[:n] + 1j * res.x0[n:]
    res.xs = [v[:n] + 1j * v[n:] for v in res.xs]
    return res
