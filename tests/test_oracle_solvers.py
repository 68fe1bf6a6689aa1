"""Pins for the oracle's FOSSILS / SPIR (CPU only).

Each test ties the oracle to a statement of the paper or to mathematics, not to itself.
"""

import os

import numpy as np
import pytest

from oracle import backward_error as be
from oracle import householder as hh
from oracle import solvers
from oracle.sketch import sketch, sketch_Ab
from synth import make_problem

U = 2.0**-52
GOLD = os.path.join(os.path.dirname(__file__), "golden", "paper_tables.txt")


def _gold():
    out = {}
    with open(GOLD) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            k1, k2, v = line.split()
            out[(k1, k2)] = float(v)
    return out


def _fe(x, P):
    return np.linalg.norm(x - P.x_true) / np.linalg.norm(P.x_true)


CASES = [(1e10, 1e-6), (1e12, 1e-3), (1e4, 1.0), (1e2, 1e-10), (1e13, 1e-8)]


@pytest.mark.parametrize("kappa,rnorm", CASES)
@pytest.mark.parametrize("method", ["fossils", "spir"])
@pytest.mark.parametrize("precond", ["qr", "svd"])
def test_backward_stable_and_forward_error_vs_qr(kappa, rnorm, method, precond):
    """Theorem 7.1 / Section 5.1: backward error at the level of Householder QR."""
    P = make_problem(4000, 50, kappa, rnorm, seed=0)
    res = solvers.solve(P.A, P.b, method, solvers.Options(precond=precond))
    xq = hh.qr_lstsq(P.A, P.b)
    bex = be.relative_backward_error(P.A, P.b, res.x, P.sigma, P.V)
    beq = be.relative_backward_error(P.A, P.b, xq, P.sigma, P.V)
    assert res.flags == 0
    assert bex <= 1e-14
    assert bex <= 30 * max(beq, U)
    # forward error within 10x of Householder QR's, floored at the Wedin scale (Fact 2.3)
    wedin = kappa * (1 + kappa * rnorm) * U
    assert _fe(res.x, P) <= 10 * max(_fe(xq, P), 0.01 * wedin)


def test_table1_residual_orthogonality_magnitude():
    """Table 1: median ||A^T(b - A x)|| ~ 4e-14 (FOSSILS), 5.3e-14 (SPIR), 5.2e-14 (QR)."""
    g = _gold()
    vals = {"fossils": [], "spir": [], "householder_qr": []}
    for seed in range(9):
        P = make_problem(4000, 50, 1e12, 1e-3, seed=100 + seed)
        for meth in ("fossils", "spir"):
            x = solvers.solve(P.A, P.b, meth, solvers.Options(seed=seed)).x
            vals[meth].append(np.linalg.norm(P.A.T @ (P.b - P.A @ x)))
        xq = hh.qr_lstsq(P.A, P.b)
        vals["householder_qr"].append(np.linalg.norm(P.A.T @ (P.b - P.A @ xq)))
    for k, v in vals.items():
        med = np.median(v)
        ref = g[("table1", k)]
        assert ref / 10 <= med <= ref * 10, (k, med, ref)
    # strongly-forward-stable methods sit four orders above; ours must not
    assert np.median(vals["fossils"]) < g[("table1", "iterative_sketching_momentum")] / 100


def test_table2_norm_of_c():
    """Table 2: ||c|| for the sketch-and-solve start ~3.0e-7 and for x_1 ~1.9e-11 (4000x50, 1e12, 1e-6)."""
    g = _gold()
    P = make_problem(4000, 50, 1e12, 1e-6, seed=1)
    res = solvers.fossils(P.A, P.b)
    c0, c1 = res.cs
    assert g[("table2", "sketch_and_solve")] / 10 <= c0 <= g[("table2", "sketch_and_solve")] * 10
    assert g[("table2", "x1")] / 10 <= c1 <= g[("table2", "x1")] * 10
    # zero initialisation: c = R^{-T} A^T b
    Y = sketch_Ab(P.A, P.b, 600, 8, 12345)
    _, Rf = hh.householder_qr(Y)
    cz = np.linalg.norm(hh.forward_substitution_transposed(Rf[:50, :50], P.A.T @ P.b))
    assert g[("table2", "zero")] / 10 <= cz <= g[("table2", "zero")] * 10


def test_spir_iteration_ceiling_figure6():
    """Figure 6 (Section 5.2): SPIR needs at most 30 iterations in total at 4000 x 50."""
    limit = _gold()[("fig6", "spir_max_total_iterations")]
    for kappa in (1e2, 1e6, 1e10, 1e13):
        for rnorm in (1e-12, 1e-6, 1e-2, 1.0):
            P = make_problem(4000, 50, kappa, rnorm, seed=7)
            res = solvers.spir(P.A, P.b)
            assert sum(res.iters) <= limit, (kappa, rnorm, res.iters)


def test_fact22_preconditioned_conditioning():
    """Fact 2.2: singular values of A R^{-1} lie in [1/(1+eta), 1/(1-eta)] (eta slack 1.5 sqrt(n/d))."""
    P = make_problem(4000, 50, 1e10, 1e-6, seed=2)
    Y = sketch(P.A, 600, 8, 12345)
    _, R = hh.householder_qr(Y)
    AR = np.linalg.solve(R.T, P.A.T).T
    s = np.linalg.svd(AR, compute_uv=False)
    eta = 1.5 * np.sqrt(50 / 600)
    assert s[-1] >= 1 / (1 + eta) and s[0] <= 1 / (1 - eta)


def test_fact69_sketch_and_solve_accuracy():
    """Fact 6.9: ||A (x - x_0)|| <~ ||b - A x|| + ||x|| u."""
    for kappa, rnorm in [(1e10, 1e-6), (1e4, 1.0), (1e12, 1e-12)]:
        P = make_problem(4000, 50, kappa, rnorm, seed=3)
        x0 = solvers.sketch_and_solve(P.A, P.b, 600)
        lhs = np.linalg.norm(P.A @ (P.x_true - x0))
        assert lhs <= 10 * (rnorm + np.linalg.norm(P.x_true) * U * 1e2)


def test_lemma73_polyak_rate():
    """Lemma 7.3 (no noise): ||dy_(j) - M^{-1} c|| <= 4 sqrt(2) j eta^{j-2} ||c||, alpha, beta optimal."""
    P = make_problem(3000, 30, 10.0, 1e-2, seed=4)
    Y = sketch(P.A, 360, 8, 9)
    _, R = hh.householder_qr(Y)
    AR = np.linalg.solve(R.T, P.A.T).T
    s = np.linalg.svd(AR, compute_uv=False)
    eta = max(1 - 1 / s[0], 1 / s[-1] - 1)          # distortion realised by this sketch
    alpha, beta = solvers.polyak_coefficients(eta)
    M = AR.T @ AR
    c = AR.T @ P.b
    ystar = np.linalg.solve(M, c)
    for j in range(1, 40):                          # the oracle's Algorithm 5 after j - 1 updates
        dy = solvers.polyak(lambda y: M @ y, c, alpha, beta, j)
        err = np.linalg.norm(dy - ystar)
        bound = 4 * np.sqrt(2) * j * eta ** (j - 2) * np.linalg.norm(c)
        assert err <= bound + 1e-13 * np.linalg.norm(ystar), j


def test_first_step_rule_special_cases():
    """Alg 4's first-step rule stops at the first iteration with ||Delta|| <= (gamma normest ||x_0|| +
    rho condest ||r_0||) u: a huge gamma stops it after one update, gamma = rho = 0 never stops it (the
    cap), and the count cannot grow with gamma."""
    P = make_problem(3000, 30, 1e8, 1e-4, seed=12)
    one = solvers.fossils(P.A, P.b, solvers.Options(gamma=1e30, steps=1))
    assert one.iters[0] == 1
    cap = solvers.fossils(P.A, P.b, solvers.Options(gamma=0.0, rho=0.0, steps=1, max_inner=37))
    assert cap.iters[0] == 37
    counts = [solvers.fossils(P.A, P.b, solvers.Options(gamma=g, steps=1)).iters[0] for g in (1e-2, 1.0, 1e2, 1e4)]
    assert all(a >= b for a, b in zip(counts, counts[1:])) and counts[0] > counts[-1], counts


def test_one_refinement_step_is_not_backward_stable():
    """Section 5.1: FOSSILS (1 step) is forward but not backward stable on hard problems."""
    P = make_problem(4000, 50, 1e12, 1e12 * U, seed=5)
    one = solvers.fossils(P.A, P.b, solvers.Options(steps=1, max_inner=100))
    two = solvers.fossils(P.A, P.b)
    b1 = be.relative_backward_error(P.A, P.b, one.x, P.sigma, P.V)
    b2 = be.relative_backward_error(P.A, P.b, two.x, P.sigma, P.V)
    assert b2 <= 1e-15 and b1 >= 30 * b2


def test_fixed_q_algorithm2():
    """Algorithm 2 with q_0 from Theorem 7.1 (eq:iterations) is backward stable."""
    P = make_problem(4000, 50, 1e10, 1e-4, seed=6)
    res = solvers.fossils(P.A, P.b, solvers.Options(fixed_q=-1))
    assert res.iters[0] == res.iters[1] == solvers.q0_theorem71(res.condest, np.sqrt(50 / 600)) - 1
    assert be.relative_backward_error(P.A, P.b, res.x, P.sigma, P.V) <= 1e-14


def test_q0_formula_values():
    eta = np.sqrt(1 / 12)
    # eq:iterations at d = 12 n
    assert solvers.q0_theorem71(1e10, eta) == 23
    assert solvers.q0_theorem71(1e14, eta) == 11
    assert solvers.q0_theorem71(1e2, eta) == 53


def test_rank_deficient_all_ones():
    """Section 4.2: an all-ones matrix must give a finite answer (truncated preconditioner)."""
    m, n = 500, 10
    A = np.ones((m, n))
    b = np.random.default_rng(0).standard_normal(m)
    for meth in ("fossils", "spir"):
        res = solvers.solve(A, b, meth)
        assert res.flags & solvers.FLAG_RANK_DEFICIENT
        assert np.all(np.isfinite(res.x)) and res.rank == 1
        # residual is the optimal one: b minus its mean
        assert abs(np.linalg.norm(b - A @ res.x) - np.linalg.norm(b - b.mean())) <= 1e-10


def test_zero_rhs_gives_zero():
    P = make_problem(400, 10, 1e3, 1e-3, seed=1)
    res = solvers.fossils(P.A, np.zeros(400))
    assert np.all(res.x == 0)


def test_first_step_rule_constants_from_text():
    """Section 4.2 text uses gamma = 1, rho = 0.04; both settings must stay backward stable."""
    P = make_problem(4000, 50, 1e10, 1e-6, seed=8)
    res = solvers.fossils(P.A, P.b, solvers.Options(gamma=1.0, rho=0.04))
    assert be.relative_backward_error(P.A, P.b, res.x, P.sigma, P.V) <= 1e-14


def test_planted_mistakes_are_caught(monkeypatch):
    """A plausible slip in the heavy-ball coefficients breaks the accuracy pins above."""
    P = make_problem(4000, 50, 1e10, 1e-6, seed=0)
    monkeypatch.setattr(solvers, "polyak_coefficients", lambda eta: ((1 - eta**2), -eta**2))
    res = solvers.fossils(P.A, P.b)
    bad = be.relative_backward_error(P.A, P.b, res.x, P.sigma, P.V)
    assert res.flags & solvers.FLAG_NOT_CONVERGED or bad > 1e-14 or sum(res.iters) > 60


def test_multi_rhs_generator_and_oracle():
    """Multi-RHS inputs: every column of B = A X + R has R perpendicular to range(A) with the
    requested norm, and the per-column oracle solves reach the backward-stable bar."""
    from synth import make_multi_problem
    P = make_multi_problem(3000, 30, 1e8, [1e-6, 1.0, 0.0], 4, seed=3)
    B, Xt = P.meta["B"], P.meta["X_true"]
    Rr = B - P.A @ Xt
    assert np.allclose(np.linalg.norm(Rr, axis=0), [1e-6, 1.0, 0.0, 1e-6], rtol=1e-6, atol=1e-12)
    assert np.max(np.abs(P.U.T @ Rr)) <= 1e-12
    res = solvers.fossils_multi(P.A, B)
    for j, r in enumerate(res):
        assert be.relative_backward_error(P.A, B[:, j], r.x, P.sigma, P.V) <= 1e-14


def test_mixed_precision_sketch_and_fallback():
    """Mixed form (sketch of the FP32 copy, FP64 refinement): sketch error bound; backward
    stable with the FP32 preconditioner while u32 condest is small; past the threshold the FP64
    sketch is used (flag); and without that fallback the FP32 preconditioner fails at kappa = 1e10
    (the single-precision reading of Lemma 6.3's hazard)."""
    from oracle.sketch import sketch_fp32
    rng = np.random.default_rng(0)
    M = rng.standard_normal((3000, 7))
    y64 = sketch(M, 300, 8, 5)
    y32 = sketch_fp32(M, 300, 8, 5)
    from oracle.sketch import sparse_sign_matrix
    S = sparse_sign_matrix(3000, 300, 8, 5)
    k = (S != 0).sum(axis=1).max()          # the longest sum (standard gamma_k bound)
    # input rounding u32 plus double-precision sums; S carries zeta^{-1/2}
    bound = 1.01 * (2.0**-24 + (k + 2) * 2.0**-53) * (abs(S) @ np.abs(M)) / np.sqrt(8)
    err = np.abs(y32 - y64)
    assert np.all(err <= bound)
    assert err.max() > 1e3 * 2.0**-53 * np.abs(y64).max()   # the input is single precision
    for kappa, flagged in [(1e3, False), (1e5, False), (1e8, True)]:
        P = make_problem(4000, 50, kappa, 1e-6, seed=3)
        r = solvers.fossils(P.A, P.b, solvers.Options(precision="mixed"))
        assert bool(r.flags & solvers.FLAG_FP64_SKETCH) == flagged, (kappa, r.flags)
        assert be.relative_backward_error(P.A, P.b, r.x, P.sigma, P.V) <= 1e-14
    P = make_problem(4000, 50, 1e10, 1e-6, seed=3)
    r = solvers.fossils(P.A, P.b, solvers.Options(precision="mixed", mixed_fallback=False))
    assert r.flags & solvers.FLAG_NOT_CONVERGED or be.relative_backward_error(P.A, P.b, r.x, P.sigma, P.V) > 1e-14


def test_lsqr_iterate_matches_scipy_lsqr_and_cg():
    """The oracle's LSQR steps against scipy's LSQR (same algorithm, exactly q iterations) and, in
    exact arithmetic, against CG on the normal equations (Section 4.3: CG and LSQR are equivalent)."""
    from scipy.sparse.linalg import lsqr
    rng = np.random.default_rng(5)
    B = rng.standard_normal((300, 20)) @ np.diag(np.logspace(0, 1, 20))  # a preconditioned-like kappa
    r = rng.standard_normal(300)
    c = B.T @ r
    # (beyond ~q = 10 the three recurrences drift apart by their own rounding: Lanczos without
    # reorthogonalization; every one of them still converges, checked at q = 60 below)
    for q in (1, 3, 6, 8):
        ys = [y for _, y, _ in solvers.lsqr_iterate(lambda v: B @ v, lambda v: B.T @ v, r, c, q)]
        ref = lsqr(B, r, atol=0, btol=0, conlim=0, iter_lim=q)[0]
        assert np.linalg.norm(ys[-1] - ref) <= 1e-12 * np.linalg.norm(ref)
        # CG on B^T B y = c from 0, q steps
        y = np.zeros(20)
        res = c.copy()
        p = c.copy()
        for _ in range(q):
            qv = B.T @ (B @ p)
            a = (res @ res) / (p @ qv)
            y = y + a * p
            rn = res - a * qv
            p = rn + (rn @ rn) / (res @ res) * p
            res = rn
        assert np.linalg.norm(ys[-1] - y) <= 1e-12 * np.linalg.norm(y)
    # q = n steps solve the problem exactly (up to rounding)
    ys = [y for _, y, _ in solvers.lsqr_iterate(lambda v: B @ v, lambda v: B.T @ v, r, c, 60)]
    assert np.linalg.norm(ys[-1] - np.linalg.lstsq(B, r, rcond=None)[0]) <= 1e-10 * np.linalg.norm(ys[-1])


@pytest.mark.parametrize("kappa,rnorm", [(1e10, 1e-6), (1e4, 1.0), (1e2, 1e-10), (1e13, 1e-8)])
@pytest.mark.parametrize("precond", ["qr", "svd"])
def test_spir_lsqr_backward_stable(kappa, rnorm, precond):
    """LSQR-based SPIR meets the same bar as the CG form (Section 4.3: similarly stable)."""
    P = make_problem(4000, 50, kappa, rnorm, seed=0)
    r = solvers.spir_lsqr(P.A, P.b, solvers.Options(precond=precond))
    assert be.relative_backward_error(P.A, P.b, r.x, P.sigma, P.V) <= 1e-14
    xq = hh.qr_lstsq(P.A, P.b)
    fe = np.linalg.norm(r.x - P.x_true) / np.linalg.norm(P.x_true)
    fq = max(np.linalg.norm(xq - P.x_true) / np.linalg.norm(P.x_true), kappa * 2.0**-52)
    assert fe <= 10 * fq
    cg = solvers.spir(P.A, P.b, solvers.Options(precond=precond))
    assert abs(r.iters[0] - cg.iters[0]) <= 2


@pytest.mark.parametrize("kappa,rnorm", [(1e12, 1e12 * U), (1e10, 1e-6)])
def test_section51_comparison_solvers(kappa, rnorm):
    """Section 5.1's comparison methods are not backward stable where FOSSILS and SPIR are:
    sketch-and-precondition from x_0 = 0 (CG or LSQR, one run) and from the sketch-and-solve start,
    and iterative sketching with momentum (FOSSILS with one refinement step)."""
    P = make_problem(4000, 50, kappa, rnorm, seed=5)
    bes, fes = {}, {}
    for name, meth, o in [("spir", "spir", {}), ("fossils", "fossils", {}),
                          ("sp_zero", "spir", dict(steps=1, init="zero")),
                          ("sp_zero_lsqr", "spir_lsqr", dict(steps=1, init="zero")),
                          ("sp_ss", "spir", dict(steps=1)), ("fossils1", "fossils", dict(steps=1))]:
        r = solvers.solve(P.A, P.b, meth, solvers.Options(**o))
        bes[name] = be.relative_backward_error(P.A, P.b, r.x, P.sigma, P.V)
        fes[name] = np.linalg.norm(r.x - P.x_true) / np.linalg.norm(P.x_true)
    assert bes["spir"] <= 1e-15 and bes["fossils"] <= 1e-15
    for k in ("sp_zero", "sp_zero_lsqr", "sp_ss", "fossils1"):
        assert bes[k] >= 30 * max(bes["spir"], bes["fossils"]), (k, bes)
    # from x_0 = 0 the method is not even forward stable (Section 5.1): its forward error is far
    # above that of the same run started from sketch-and-solve
    assert fes["sp_zero"] >= 100 * fes["sp_ss"], fes
