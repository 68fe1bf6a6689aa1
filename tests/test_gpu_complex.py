"""Complex least squares on the GPU (fossils_solve_complex / spir_solve_complex through the C ABI).

Bar (the same as the real path): relative KW backward error <= 1e-14 and forward error within 10x
of complex Householder QR's (floored at kappa u); iteration counts close to the oracle's complex
solver (FOSSILS/SPIR on the realification); on a Prony problem (Appendix B) the solution agrees
with complex Householder QR's to condest u.
"""

import numpy as np
import pytest

from gpu_util import assert_stats, host
from oracle import backward_error as be
from oracle import householder as hh
from oracle import solvers
from synth import make_complex_problem, make_prony_problem

pytestmark = pytest.mark.gpu
U = 2.0**-52


@pytest.fixture(scope="module")
def ctx():
    from paper_2406_03468_amd import binding
    c = binding.Context(0)
    yield c
    c.close()


def dev_cmat(M, ld=None):
    """numpy complex (rows, cols) -> torch complex128 cuda tensor, column-major with leading dimension ld
    (padding rows NaN)."""
    import torch
    M = np.asarray(M, dtype=np.complex128)
    rows, cols = M.shape
    ld = ld or rows
    buf = torch.full((cols, ld), complex("nan+nanj"), dtype=torch.complex128, device="cuda")
    buf[:, :rows] = torch.as_tensor(np.ascontiguousarray(M.T), device="cuda")
    return buf.t()[:rows, :]


def dev_cvec(v):
    import torch
    return torch.as_tensor(np.asarray(v, dtype=np.complex128)).to("cuda")


def _solve(ctx, A, b, method="fossils", ld=None, **kw):
    import torch
    from paper_2406_03468_amd import binding
    m, n = A.shape
    o = binding.fs_options_default(2 * m, 2 * n)
    o.precond = binding.FS_PRECOND_SVD
    for k, v in kw.items():
        setattr(o, k, v)
    x = torch.zeros(n, dtype=torch.complex128, device="cuda")
    st, info = binding.fossils_solve_complex(ctx, dev_cmat(A, ld), dev_cvec(b), x, o, method=method)
    return st, info, host(x)


def _fe(x, xt):
    return np.linalg.norm(x - xt) / np.linalg.norm(xt)


@pytest.mark.parametrize("method", ["fossils", "spir"])
@pytest.mark.parametrize("kappa,rnorm", [(1e2, 1.0), (1e6, 1e-4), (1e10, 1e-8), (1e12, 1e-3)])
def test_complex_solve_vs_oracle(ctx, method, kappa, rnorm):
    P = make_complex_problem(4000, 40, kappa, rnorm, seed=1)
    st, info, x = _solve(ctx, P.A, P.b, method, ld=4003)
    floor = kappa >= 1e12 and method == "spir"   # see the C1 parity test of the real path
    assert st == 0 or (floor and st == 2), info.to_dict()
    assert be.relative_backward_error_complex(P.A, P.b, x, P.sigma, P.V) <= 1e-14
    xq = hh.qr_lstsq_complex(P.A, P.b)
    fq = max(_fe(xq, P.x_true), kappa * U)
    assert _fe(x, P.x_true) <= 10 * fq, (_fe(x, P.x_true), fq)
    ref = solvers.solve_complex(P.A, P.b, method, solvers.Options(precond="svd"))
    assert abs(info.iters[0] - ref.iters[0]) <= 3, (list(info.iters), ref.iters)
    if not floor:
        assert abs(info.iters[1] - ref.iters[1]) <= 5, (list(info.iters), ref.iters)
    # the realified sketch's statistics: every singular value twice, the same condest scale
    assert_stats(info, ref.condest, rel=1e-9 + 1e3 * ref.condest * U)
    assert np.linalg.norm(x - ref.x) <= 10 * fq * np.linalg.norm(P.x_true)


@pytest.mark.parametrize("m,n,K", [(20000, 100, 10), (6001, 37, 5)])
def test_prony_problem(ctx, m, n, K):
    """The first least-squares solve of Prony's method (Appendix B), noise 1e-6."""
    P = make_prony_problem(m, n, K, 1e-6, seed=2)
    st, info, x = _solve(ctx, P.A, P.b, "fossils")
    assert st == 0, info.to_dict()
    assert 1e5 <= info.condest <= 1e8, info.condest   # the paper's Prony problems: about 1e6
    assert be.relative_backward_error_complex(P.A, P.b, x) <= 1e-14
    xq = hh.qr_lstsq_complex(P.A, P.b)
    assert np.linalg.norm(x - xq) <= 10 * info.condest * U * np.linalg.norm(xq)


def test_real_valued_input(ctx):
    """A complex problem with real A and b: the imaginary part of x is (numerically) zero and the real
    part solves the real problem."""
    from synth import make_problem
    P = make_problem(3000, 30, 1e6, 1e-5, seed=3)
    st, info, x = _solve(ctx, P.A.astype(np.complex128), P.b.astype(np.complex128))
    assert st == 0
    xq = hh.qr_lstsq(P.A, P.b)
    fq = max(_fe(xq, P.x_true), P.kappa * U)
    assert np.linalg.norm(x.imag) <= 10 * fq * np.linalg.norm(P.x_true)
    assert _fe(x.real, P.x_true) <= 10 * fq
    assert be.relative_backward_error(P.A, P.b, x.real, P.sigma, P.V) <= 1e-14


@pytest.mark.parametrize("m,n", [(50, 50), (700, 1)])
def test_edge_shapes(ctx, m, n):
    """A square system and a single column."""
    P = make_complex_problem(m, n, 1e3, 0.0 if m == n else 1e-2, seed=4)
    st, info, x = _solve(ctx, P.A, P.b, ld=m + 1)
    assert st == 0, info.to_dict()
    xq = hh.qr_lstsq_complex(P.A, P.b)
    fq = max(_fe(xq, P.x_true), 1e3 * U)
    assert _fe(x, P.x_true) <= 10 * fq


def test_zero_rhs_and_argument_errors(ctx):
    import ctypes
    import torch
    from paper_2406_03468_amd import binding
    P = make_complex_problem(500, 10, 10.0, 1e-2, seed=5)
    st, info, x = _solve(ctx, P.A, np.zeros(500, dtype=np.complex128))
    assert st == 0 and np.all(x == 0)
    lib = binding.load()
    A = dev_cmat(P.A)
    b = dev_cvec(P.b)
    xo = torch.zeros(10, dtype=torch.complex128, device="cuda")
    c = ctypes.c_void_p
    # misaligned (8-byte offset) pointers and a short leading dimension are refused before device work
    assert lib.fossils_solve_complex(ctx.h, 500, 10, c(A.data_ptr() + 8), 500, c(b.data_ptr()), c(xo.data_ptr()),
                                     None, None) == binding.FS_ERR_INVALID_ARG
    assert lib.fossils_solve_complex(ctx.h, 500, 10, c(A.data_ptr()), 499, c(b.data_ptr()), c(xo.data_ptr()),
                                     None, None) == binding.FS_ERR_SHAPE
    assert lib.spir_solve_complex(ctx.h, 5, 10, c(A.data_ptr()), 500, c(b.data_ptr()), c(xo.data_ptr()),
                                  None, None) == binding.FS_ERR_SHAPE
