"""GPU parity of each hot-path step against the CPU oracle, through the C ABI."""

import numpy as np
import pytest

from gpu_util import dev_colmajor, dev_vec, empty_colmajor, host
from oracle import householder as hh
from oracle import philox
from oracle import sketch as osk

pytestmark = pytest.mark.gpu
U = 2.0**-52


@pytest.fixture(scope="module")
def ctx():
    from paper_2406_03468_amd import binding
    c = binding.Context(0)
    yield c
    c.close()


# ---------------------------------------------------------------- sketch indices (bit exact)
@pytest.mark.parametrize("m,d,zeta,seed", [(100003, 600, 8, 12345), (50001, 12000, 8, 7), (3001, 40000, 8, 99),
                                           (20000, 37, 5, 2**40 + 3), (4096, 300, 64, 1), (777, 8, 8, 5),
                                           (1000, 1, 1, 0)])
def test_sketch_indices_bit_exact(ctx, m, d, zeta, seed):
    from paper_2406_03468_amd import binding
    sk = binding.sketch_create(ctx, m, d, zeta, seed)
    try:
        rows, signs = binding.sketch_indices(sk, 0, m)
        rw, sw = binding.sketch_indices(sk, m // 3, 17)
    finally:
        sk.close()
    r0, s0 = philox.sparse_sign_indices(m, d, zeta, seed)
    assert np.array_equal(rows, r0)
    assert np.array_equal(signs, s0)
    assert np.array_equal(rw, r0[m // 3: m // 3 + 17])


def test_sketch_indices_full_size_bit_exact(ctx):
    """All m*zeta = 8e6 positions and signs at m = 1e6, d = 12000."""
    from paper_2406_03468_amd import binding
    m, d, zeta, seed = 1_000_000, 12000, 8, 12345
    sk = binding.sketch_create(ctx, m, d, zeta, seed)
    try:
        rows, signs = binding.sketch_indices(sk, 0, m)
    finally:
        sk.close()
    r0, s0 = philox.sparse_sign_indices(m, d, zeta, seed)
    assert np.array_equal(rows, r0) and np.array_equal(signs, s0)


# ---------------------------------------------------------------- sketch apply
@pytest.mark.parametrize("m,n,d,scale", [(20011, 37, 450, False), (20011, 37, 450, True), (30001, 300, 3600, True),
                                         (9001, 5, 24000, True), (5000, 1, 12, False)])
def test_sketch_apply_matches_oracle(ctx, m, n, d, scale):
    from paper_2406_03468_amd import binding
    rng = np.random.default_rng(m + n)
    A = rng.standard_normal((m, n)) * rng.uniform(0.1, 10, size=n)
    b = rng.standard_normal(m)
    sk = binding.sketch_create(ctx, m, d, 8, 4242)
    try:
        Ad, bd = dev_colmajor(A, ld=m + 3), dev_vec(b)
        Y = empty_colmajor(d, n + 1, ld=d + 1)
        cn = dev_vec(np.zeros(n))
        binding.sketch_apply(sk, Ad, bd, Y, cn, scale_columns=scale)
    finally:
        sk.close()
    norms = np.linalg.norm(A, axis=0)
    As = A / norms if scale else A
    M = np.column_stack([As, b])
    Yr = osk.sketch_Ab(As, b, d, 8, 4242)
    Yg = host(Y)
    # error bound per entry: (terms in the row) * u * sum |terms| for the summation in any order,
    # plus ~10 u for the column scale (norm accumulated in another order, sqrt, two divisions)
    S = osk.sparse_sign_matrix(m, d, 8, 4242)
    absS = abs(S)
    hits = np.asarray(absS.sum(axis=1)).ravel()
    sum_abs = (absS @ np.abs(M)) / np.sqrt(8)
    bound = (hits[:, None] + 10) * U * sum_abs
    assert np.all(np.abs(Yg - Yr) <= bound)
    assert np.allclose(host(cn), norms**2, rtol=1e-13, atol=0)


# ---------------------------------------------------------------- QR of the sketch
@pytest.mark.parametrize("d,k", [(600, 51), (3600, 301), (1000, 33), (64, 64), (130, 1), (128, 64), (4096, 96)])
def test_qr_matches_householder_oracle(ctx, d, k):
    """(k a multiple of the 32-column panel: the last panel has no trailing update.)"""
    from paper_2406_03468_amd import binding
    rng = np.random.default_rng(d * 7 + k)
    Y0 = rng.standard_normal((d, k))
    Y = dev_colmajor(Y0, ld=d + 5)
    binding.fs_sketch_qr(ctx, Y)
    Rg = np.triu(host(Y)[:k, :k])
    _, Rr = hh.householder_qr(Y0)
    assert np.all(np.diag(Rg) >= 0)
    nrm = np.linalg.norm(Y0)
    assert np.max(np.abs(Rg - Rr)) <= 200 * U * nrm * np.linalg.cond(Y0)


@pytest.mark.parametrize("d,k,kappa", [(600, 51, 1e10), (12000, 1001, 1e12)])
def test_qr_backward_property_ill_conditioned(ctx, d, k, kappa):
    """R^T R = Y^T Y up to O(u ||Y||^2) for any conditioning (Householder is backward stable)."""
    from paper_2406_03468_amd import binding
    rng = np.random.default_rng(1)
    Q1, _ = np.linalg.qr(rng.standard_normal((d, k)))
    Q2, _ = np.linalg.qr(rng.standard_normal((k, k)))
    Y0 = (Q1 * 10.0 ** -np.linspace(0, np.log10(kappa), k)) @ Q2.T
    Y = dev_colmajor(Y0)
    binding.fs_sketch_qr(ctx, Y)
    Rg = np.triu(host(Y)[:k, :k])
    err = np.linalg.norm(Rg.T @ Rg - Y0.T @ Y0) / np.linalg.norm(Y0) ** 2
    assert err <= 50 * np.sqrt(d) * U


# ---------------------------------------------------------------- SVD of R
@pytest.mark.parametrize("n,kappa", [(50, 1e10), (301, 1e12), (7, 1.0), (1000, 1e10), (1999, 1e6), (130, 1e14),
                                     (1000, 1e14), (300, 1e13), (200, 1e10), (256, 1e12), (97, 1e8),
                                     (65, 1e12), (111, 1e14), (128, 1e10)])
def test_svd_of_triangular(ctx, n, kappa):
    from paper_2406_03468_amd import binding
    rng = np.random.default_rng(n)
    Q1, _ = np.linalg.qr(rng.standard_normal((n, n)))
    Q2, _ = np.linalg.qr(rng.standard_normal((n, n)))
    s = 10.0 ** -np.linspace(0, np.log10(kappa), n)
    R = np.linalg.qr((Q1 * s) @ Q2.T, mode="r")
    R = R * np.where(np.diag(R) < 0, -1.0, 1.0)[:, None]
    Rd = dev_colmajor(R)
    sig = dev_vec(np.zeros(n))
    V = empty_colmajor(n, n)
    sweeps = binding.fs_svd_triangular(ctx, Rd, sig, V)
    sg, Vg = host(sig), host(V)
    sr = np.linalg.svd(R, compute_uv=False)
    assert np.all(np.diff(sg) <= 0)
    assert np.all(np.abs(sg - sr) <= 1e-13 * sr[0] + 1e-9 * sr)
    assert np.linalg.norm(Vg.T @ Vg - np.eye(n)) <= 1e-12 * n
    assert np.linalg.norm(R.T @ R - (Vg * sg**2) @ Vg.T) <= 1e-13 * n * sr[0] ** 2
    assert 1 <= sweeps <= 40
    # V is orthogonal to working precision (not only to the Jacobi tolerance n u), so the
    # preconditioner V Sigma^{-1} keeps R V Sigma^{-1} orthogonal up to O(1) even at condest 1e14
    # (the normalized Jacobi columns alone give cond up to ~condest n u: ~20 at n = 1000, 1e14)
    assert np.abs(Vg.T @ Vg - np.eye(n)).max() <= 4 * U * np.sqrt(n)
    assert np.linalg.cond(R @ (Vg / sg)) <= 1.2


# ---------------------------------------------------------------- fused passes
PASS_SHAPES = [(10007, 1), (10007, 7), (10007, 50), (10007, 64), (10007, 65), (10007, 300), (20011, 1000),
               (4099, 1025), (3001, 2100), (2001, 4500), (64, 16)]


def _pass_bound(A, z):
    return (A.shape[0] + A.shape[1]) * U * (np.abs(A).T @ (np.abs(A) @ np.abs(z))) * 4


@pytest.mark.parametrize("m,n", PASS_SHAPES)
def test_normal_pass_matches_oracle(ctx, m, n):
    from oracle.solvers import normal_pass
    from paper_2406_03468_amd import binding
    rng = np.random.default_rng(m + 3 * n)
    A = rng.standard_normal((m, n))
    z = rng.standard_normal(n)
    v = dev_vec(np.zeros(n))
    binding.fs_normal_pass(ctx, dev_colmajor(A), dev_vec(z), v)
    assert np.all(np.abs(host(v) - normal_pass(A, z)) <= _pass_bound(A, z))


@pytest.mark.parametrize("m,n,ld", [(10007, 50, 10008), (10007, 50, 10009), (999, 33, 2000)])
def test_normal_pass_leading_dimension(ctx, m, n, ld):
    from oracle.solvers import normal_pass
    from paper_2406_03468_amd import binding
    rng = np.random.default_rng(ld)
    A = rng.standard_normal((m, n))
    z = rng.standard_normal(n)
    v = dev_vec(np.zeros(n))
    binding.fs_normal_pass(ctx, dev_colmajor(A, ld=ld), dev_vec(z), v)
    assert np.all(np.abs(host(v) - normal_pass(A, z)) <= _pass_bound(A, z))


@pytest.mark.parametrize("m,n", [(10007, 50), (20011, 1000), (5, 3)])
def test_residual_pass_matches_oracle(ctx, m, n):
    from oracle.solvers import residual_pass
    from paper_2406_03468_amd import binding
    rng = np.random.default_rng(m + n)
    A = rng.standard_normal((m, n))
    x = rng.standard_normal(n)
    b = A @ x + 1e-3 * rng.standard_normal(m)
    g = dev_vec(np.zeros(n))
    r2 = binding.fs_residual_pass(ctx, dev_colmajor(A), dev_vec(b), dev_vec(x), g)
    gr, r2r = residual_pass(A, b, x)
    bound = (m + n) * U * (np.abs(A).T @ (np.abs(b) + np.abs(A) @ np.abs(x))) * 4
    assert np.all(np.abs(host(g) - gr) <= bound)
    assert abs(r2 - r2r) <= 1e-10 * r2r + 1e-12 * np.linalg.norm(b) ** 2


def _nan_fenced(A, ld, extra_cols):
    """A inside a device buffer whose padding rows (m..ld-1) and trailing columns are NaN: any read
    outside A shows up as NaN in the result instead of touching foreign memory."""
    import torch
    m, n = A.shape
    buf = torch.full((n + extra_cols, ld), float("nan"), dtype=torch.float64, device="cuda")
    buf[:n, :m] = torch.as_tensor(np.ascontiguousarray(A.T), device="cuda")
    return buf[:n, :m].t()  # (m, n) view, column-major, leading dimension ld


# n chosen so that ceil(n / columns-per-round) falls between the powers of two for every tile
# height (65..97 -> 3 slots at H = 32, 130/150 -> 5, 300 -> 5 at H = 16, 700 -> 11, 1500 -> 12, 2100 -> 9)
FENCE_SHAPES = [(6001, 20, 0), (6001, 65, 0), (6001, 97, 2), (5003, 130, 1), (5003, 150, 0), (4001, 300, 3),
                (4001, 700, 0), (3001, 1500, 1), (2500, 2100, 0)]


@pytest.mark.parametrize("m,n,pad", FENCE_SHAPES)
def test_passes_stay_inside_A(ctx, m, n, pad):
    from oracle.solvers import normal_pass, residual_pass
    from paper_2406_03468_amd import binding
    rng = np.random.default_rng(n)
    A = rng.standard_normal((m, n))
    z = rng.standard_normal(n)
    b = A @ z + rng.standard_normal(m)
    Ad = _nan_fenced(A, m + pad, extra_cols=300)
    v = dev_vec(np.zeros(n))
    binding.fs_normal_pass(ctx, Ad, dev_vec(z), v)
    vh = host(v)
    assert np.all(np.isfinite(vh))
    assert np.all(np.abs(vh - normal_pass(A, z)) <= _pass_bound(A, z))
    g = dev_vec(np.zeros(n))
    r2 = binding.fs_residual_pass(ctx, Ad, dev_vec(b), dev_vec(z), g)
    gr, r2r = residual_pass(A, b, z)
    assert np.all(np.isfinite(host(g))) and np.isfinite(r2)
    assert abs(r2 - r2r) <= 1e-10 * r2r


def test_normal_pass_full_size(ctx):
    """The launch configuration of the 1e6 x 1000 solve, against numpy on the host."""
    import torch
    from paper_2406_03468_amd import binding
    m, n = 1_000_000, 1000
    gen = torch.Generator(device="cuda")
    gen.manual_seed(5)
    At = torch.randn((n, m), generator=gen, dtype=torch.float64, device="cuda")
    A = At.t()
    z = torch.randn((n,), generator=gen, dtype=torch.float64, device="cuda")
    v = torch.zeros(n, dtype=torch.float64, device="cuda")
    binding.fs_normal_pass(ctx, A, z, v)
    Ah = host(At).T
    zh = host(z)
    ref = Ah.T @ (Ah @ zh)
    bound = 4 * (m + n) * U * (np.abs(Ah).T @ (np.abs(Ah) @ np.abs(zh)))
    assert np.all(np.abs(host(v) - ref) <= bound)


# ---------------------------------------------------------------- triangular solves
@pytest.mark.parametrize("n", [1, 50, 64, 65, 300, 1000])
@pytest.mark.parametrize("transpose", [False, True])
def test_trsv_matches_substitution(ctx, n, transpose):
    from paper_2406_03468_amd import binding
    rng = np.random.default_rng(n)
    R = np.triu(rng.standard_normal((n, n))) + 4 * np.sqrt(n) * np.eye(n)
    y = rng.standard_normal(n)
    x = dev_vec(np.zeros(n))
    binding.fs_trsv(ctx, dev_colmajor(R, ld=n + 2), dev_vec(y), x, transpose=transpose)
    ref = hh.forward_substitution_transposed(R, y) if transpose else hh.back_substitution(R, y)
    assert np.allclose(host(x), ref, rtol=1e-12, atol=1e-14)


# ---------------------------------------------------------------- explicit inverse of R
@pytest.mark.parametrize("n,kappa", [(1, 1.0), (5, 1e2), (64, 1e4), (65, 1e6), (127, 1e8), (200, 1e10),
                                     (333, 1e12), (333, 1e14), (513, 1e10), (1000, 1e10), (1500, 1e8)])
def test_triangular_inverse_matches_substitution(ctx, n, kappa):
    """X = R^{-1} column by column against the oracle's back substitution of R x = e_c, within the
    forward-error bound of a triangular inverse, |X^ - X| <= c n u |X| |R| |X| (normwise per column,
    c = 1); zeros below the diagonal and 1 / r_ii on it exactly.  R is the R factor of a matrix with
    geometric singular values, stored with ld > n and other data below its diagonal (as in the
    sketch, whose lower part holds reflectors)."""
    from paper_2406_03468_amd import binding
    rng = np.random.default_rng(n + int(np.log10(kappa)))
    G = rng.standard_normal((2 * n + 3, n)) * np.logspace(0, -np.log10(kappa), n)
    Ru = np.triu(np.linalg.qr(G, mode="r"))
    Rs = Ru + np.tril(rng.standard_normal((n, n)), -1)
    X = empty_colmajor(n, n)
    binding.fs_triangular_inverse(ctx, dev_colmajor(Rs, ld=n + 5), X)
    Xg = host(X)
    assert np.all(np.tril(Xg, -1) == 0.0)
    assert np.array_equal(np.diag(Xg), 1.0 / np.diag(Ru))
    edges = {0, 1, 62, 63, 64, 65, 127, 128, 500, 511, 512, 513, 767, 768, 958, 959, 960, 998, 999, 1023, 1024,
             1025, 1499}
    cols = list(range(n)) if n <= 333 else sorted({c for c in edges if c < n}
                                                  | set(rng.choice(n, 16, replace=False).tolist()))
    M = np.abs(Xg) @ np.abs(Ru) @ np.abs(Xg)
    for c in cols:
        e = np.zeros(n)
        e[c] = 1.0
        ref = hh.back_substitution(Ru, e)
        assert np.linalg.norm(Xg[:, c] - ref) <= n * U * np.linalg.norm(M[:, c]), c
