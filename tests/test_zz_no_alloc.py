"""fossils_solve_noalloc (the entry point whose workspace is the library's file-scope device array,
for callers that cannot allocate) against fossils_solve, through the C ABI: two calls in a row,
the second on a smaller problem, each meeting the bar (backward error <= 1e-14, forward error within
10x of Householder QR's) and agreeing with the allocating entry point's solution to the forward-error
scale (not bitwise: the sketch's sums use device atomics in a run-dependent order)."""

import ctypes

import numpy as np
import pytest

from gpu_util import dev_colmajor, dev_vec, host
from oracle import backward_error as be
from oracle import householder as hh
from synth import make_problem

pytestmark = pytest.mark.gpu
U = 2.0**-52


@pytest.fixture(scope="module")
def ctx():
    from paper_2406_03468_amd import binding
    c = binding.Context(0)
    yield c
    c.close()


def _noalloc(ctx, A, b, x, opts):
    """Straight through the C ABI (the loaded library's entry point, plain pointers)."""
    from paper_2406_03468_amd import binding
    fn = binding.load().fossils_solve_noalloc
    m, n = A.shape
    info = binding.FsInfo()
    st = fn(ctx.h, m, n, A.data_ptr(), A.stride(1), b.data_ptr(), x.data_ptr(), ctypes.byref(opts),
            ctypes.byref(info))
    return st, info


def _fe(x, P):
    return np.linalg.norm(x - P.x_true) / np.linalg.norm(P.x_true)


def test_noalloc_matches_fossils_solve(ctx):
    import torch
    from paper_2406_03468_amd import binding
    for (m, n, kappa, rn, seed) in [(20011, 300, 1e10, 1e-6, 3), (4000, 50, 1e12, 1e-3, 4)]:
        P = make_problem(m, n, kappa, rn, seed=seed)
        A, b = dev_colmajor(P.A), dev_vec(P.b)
        o = binding.fs_options_default(m, n)
        o.overlap_svd = 0  # the schedule the no-alloc entry point runs
        x_ref = torch.zeros(n, dtype=torch.float64, device="cuda")
        st_ref, info_ref = binding.fossils_solve(ctx, A, b, x_ref, o)
        x = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
        st, info = _noalloc(ctx, A, b, x, o)
        torch.cuda.synchronize()
        assert st == st_ref == 0, (st, st_ref, info.to_dict())
        xh, xr = host(x), host(x_ref)
        xq = hh.qr_lstsq(P.A, P.b)
        ref = max(_fe(xq, P), _fe(xr, P), kappa * U)
        assert be.relative_backward_error(P.A, P.b, xh, P.sigma, P.V) <= 1e-14
        assert _fe(xh, P) <= 10 * max(_fe(xq, P), kappa * U)
        assert np.linalg.norm(xh - xr) / np.linalg.norm(P.x_true) <= 10 * ref
        assert abs(info.iters[0] - info_ref.iters[0]) <= 2 and abs(info.iters[1] - info_ref.iters[1]) <= 5
        # condest moves with the rounding of the sketch's atomic sums: |d sigma_min| <~ u ||S A||_F
        assert abs(info.condest - info_ref.condest) <= 50 * U * np.sqrt(n) * info_ref.condest ** 2 + 1e-10 * info_ref.condest


def test_noalloc_rejects_sizes_beyond_its_array(ctx):
    import torch
    from paper_2406_03468_amd import binding
    m, n = 40000, 2000  # sketch alone 8 * 24000 * 2001 bytes = 384 MB
    A = torch.zeros((n, m), dtype=torch.float64, device="cuda").t()
    b = torch.zeros(m, dtype=torch.float64, device="cuda")
    x = torch.zeros(n, dtype=torch.float64, device="cuda")
    st, _ = _noalloc(ctx, A, b, x, binding.fs_options_default(m, n))
    assert st == binding.FS_ERR_TOO_LARGE
