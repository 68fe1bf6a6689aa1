"""Pins for the oracle's backward-error tools (CPU only)."""

import numpy as np
import pytest

from oracle import backward_error as be
from oracle import sketch
from synth import make_problem


def _tiny(seed, m=9, n=3):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((m, n)) @ np.diag([1.0, 1e-2, 1e-4][:n])
    b = rng.standard_normal(m)
    x = np.linalg.lstsq(A, b, rcond=None)[0] + 1e-3 * rng.standard_normal(n)
    return A, b, x


@pytest.mark.parametrize("seed", range(12))
@pytest.mark.parametrize("theta", [1.0, 10.0, np.inf])
def test_kw_brackets_exact_backward_error(seed, theta):
    """Fact 4.1: KW <= BE <= sqrt(2) KW."""
    A, b, x = _tiny(seed)
    e = be.exact_backward_error(A, b, x, theta)
    k = be.kw_estimate(A, b, x, theta)
    assert k <= e * (1 + 1e-8) + 1e-15
    assert e <= np.sqrt(2) * k * (1 + 1e-8) + 1e-15


def test_exact_backward_error_vanishes_at_ls_solution():
    rng = np.random.default_rng(0)
    A = rng.standard_normal((7, 3))
    b = rng.standard_normal(7)
    x = np.linalg.lstsq(A, b, rcond=None)[0]
    assert be.exact_backward_error(A, b, x, 1.0) <= 1e-7 * np.linalg.norm(A)
    # a consistent system solved exactly has zero backward error too
    assert be.exact_backward_error(A, A @ x, x, 1.0) <= 1e-7


def test_exact_backward_error_upper_bound_by_explicit_perturbation():
    """dA = r x^T / ||x||^2 makes x exact for (A + dA) x = b, so BE_inf <= ||r|| / ||x||."""
    A, b, x = _tiny(3)
    r = b - A @ x
    assert be.exact_backward_error(A, b, x, np.inf) <= np.linalg.norm(r) / np.linalg.norm(x) * (1 + 1e-12)


@pytest.mark.parametrize("seed", range(4))
def test_kw_svd_form_matches_literal_form(seed):
    A, b, x = _tiny(seed, m=12, n=3)
    for theta in (0.5, 3.0):
        a = be.kw_estimate(A, b, x, theta)
        c = be.kw_estimate_dense(A, b, x, theta)
        assert abs(a - c) <= 1e-9 * c


def test_known_svd_kw_matches_full_kw():
    P = make_problem(400, 10, 1e6, 1e-5, seed=2)
    x = np.linalg.lstsq(P.A, P.b, rcond=None)[0] * (1 + 1e-9)
    theta = np.linalg.norm(P.A) / np.linalg.norm(P.b)
    k1 = be.kw_known_svd(P.A, P.b, x, P.sigma, P.V, theta)
    k2 = be.kw_estimate(P.A, P.b, x, theta)
    assert abs(k1 - k2) <= 1e-3 * k2


@pytest.mark.parametrize("seed", range(4))
def test_sketched_kw_within_proposition_42(seed):
    """(1 - eta) KW_sk <= BE <= sqrt(2) (1 + eta) KW_sk with eta the sketch's distortion."""
    rng = np.random.default_rng(seed)
    m, n, d = 60, 4, 40
    A = rng.standard_normal((m, n)) @ np.diag([1.0, 0.3, 1e-2, 1e-3])
    b = rng.standard_normal(m)
    x = np.linalg.lstsq(A, b, rcond=None)[0] + 1e-4 * rng.standard_normal(n)
    SA = sketch.sketch(A, d, 8, 100 + seed)
    _, s, Vt = np.linalg.svd(SA, full_matrices=False)
    Q, _ = np.linalg.qr(A)
    sq = np.linalg.svd(sketch.sketch(Q, d, 8, 100 + seed), compute_uv=False)
    eta = max(sq[0] - 1, 1 - sq[-1])
    theta = 1.0
    ksk = be.sketched_kw(A, b, x, s, Vt.T, theta)
    e = be.exact_backward_error(A, b, x, theta)
    assert (1 - eta) * ksk <= e * (1 + 1e-8)
    assert e <= np.sqrt(2) * (1 + eta) * ksk * (1 + 1e-8)
