"""fossils_solve_batched on the GPU: many independent problems of uneven shapes, set up on several
streams and refined in lockstep (one launch per phase for the whole batch).  Each problem's x must
meet the single-solve bar and agree with its own fossils_solve (serial order, the same options) to the
forward-error scale; the iteration counts agree up to the rounding of the sums (the batched passes
share a problem's rows among a different number of work-groups, and the sketch's atomic sums are
accumulated in a run-dependent order)."""

import numpy as np
import pytest

from gpu_util import dev_colmajor, dev_vec, host
from oracle import backward_error as be
from oracle import householder as hh
from oracle import solvers
from synth import make_problem

pytestmark = pytest.mark.gpu
U = 2.0**-52


@pytest.fixture(scope="module")
def ctx():
    from paper_2406_03468_amd import binding
    c = binding.Context(0)
    yield c
    c.close()


def _mix(seed, count, nmax=300, mmax=40000):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(rng.integers(8, nmax))
        m = int(rng.integers(max(20 * n, 1000), mmax))
        kappa = 10.0 ** rng.uniform(1, 12)
        rn = 10.0 ** rng.uniform(-12, 0)
        out.append(make_problem(m, n, kappa, rn, seed=1000 * seed + i))
    return out


def _solo(ctx, A, b, n, overlap=0, method="fossils"):
    import torch
    from paper_2406_03468_amd import binding
    o = binding.fs_options_default(A.shape[0], n)
    o.overlap_svd = overlap
    x = torch.zeros(n, dtype=torch.float64, device="cuda")
    st, info = (binding.spir_solve if method == "spir" else binding.fossils_solve)(ctx, A, b, x, o)
    return st, info, host(x)


def _check_pair(P, x_b, x_s, ib, is_, sb, ss, tag, same_order=True, qr=hh.qr_lstsq):
    """Batched result (x_b, info ib, status sb) against fossils_solve's (x_s, is_, ss).  same_order: both
    ran in the serial order (else the batch's fallback ran with the SVD beside the first step, whose
    timing decides where the steps stop: only the bar, the agreement of x and the statistics)."""
    from paper_2406_03468_amd import binding
    assert sb == ss, (tag, sb, ss)
    bb = be.relative_backward_error(P.A, P.b, x_b, P.sigma, P.V)
    bs = be.relative_backward_error(P.A, P.b, x_s, P.sigma, P.V)
    assert bb <= 1e-14 and bs <= 1e-14, (tag, bb, bs, ib.to_dict())
    xq = qr(P.A, P.b)
    ref = max(np.linalg.norm(v - P.x_true) / np.linalg.norm(P.x_true) for v in (xq, x_s))
    ref = max(ref, P.kappa * U)
    assert np.linalg.norm(x_b - x_s) / np.linalg.norm(P.x_true) <= 10 * ref, (tag, P.kappa, ref)
    cs = is_.condest
    if ib.flags & binding.FS_FLAG_SVD_ABANDONED:  # stopped before the SVD: lower bounds within 4x
        assert cs / 4 <= ib.condest <= cs * (1 + 1e-6), (tag, ib.condest, cs)
    else:
        assert abs(ib.condest - cs) <= 50 * U * np.sqrt(P.A.shape[1]) * cs**2 + 1e-10 * cs, (tag, ib.condest, cs)
    if not same_order:
        return
    assert abs(ib.iters[0] - is_.iters[0]) <= 2, (tag, ib.iters, is_.iters)
    if P.kappa < 1e12:
        assert abs(ib.iters[1] - is_.iters[1]) <= 5, (tag, ib.iters, is_.iters)
    assert (ib.flags & binding.FS_FLAG_NOT_CONVERGED) == (is_.flags & binding.FS_FLAG_NOT_CONVERGED) or \
        P.kappa >= 1e11, (tag, ib.flags, is_.flags)


@pytest.mark.parametrize("seed,count,method", [(1, 6, "fossils"), (4, 6, "spir"), (2, 24, "alternate"),
                                               (3, 16, "spir")])
def test_batched_matches_solo(ctx, seed, count, method):
    """FOSSILS, SPIR, or the two alternating inside one batch."""
    import torch
    from paper_2406_03468_amd import binding
    probs = _mix(seed, count)
    dev = [(dev_colmajor(P.A), dev_vec(P.b), torch.full((P.A.shape[1],), np.nan, dtype=torch.float64, device="cuda"))
           for P in probs]
    torch.cuda.synchronize()
    meths = [(("fossils", "spir")[i % 2] if method == "alternate" else method) for i in range(count)]
    print("batched:", method, "seed", seed, "count", count, [P.A.shape for P in probs], flush=True)
    s, sts, infos = binding.fossils_solve_batched(ctx, [(A, b, x, mt) for (A, b, x), mt in zip(dev, meths)])
    assert s in (0, binding.FS_WARN_NOT_CONVERGED), sts
    for i, (P, (A, b, x)) in enumerate(zip(probs, dev)):
        ss, si, xs = _solo(ctx, A, b, P.A.shape[1], method=meths[i])
        assert infos[i].phase_ms[0] > 0 and infos[i].phase_ms[4] > 0
        _check_pair(P, host(x), xs, infos[i], si, sts[i], ss, (seed, i, P.A.shape, P.kappa, P.resid_norm))
        if count <= 6:
            # and against the oracle's run of the same method (Algorithm 4 with the SVD preconditioner)
            ref = solvers.solve(P.A, P.b, meths[i], solvers.Options(precond="svd"))
            xb = host(x)
            fq = max(np.linalg.norm(hh.qr_lstsq(P.A, P.b) - P.x_true) / np.linalg.norm(P.x_true), P.kappa * U)
            assert np.linalg.norm(xb - ref.x) / np.linalg.norm(P.x_true) <= 10 * fq, (seed, i, "oracle")
            assert abs(infos[i].iters[0] - ref.iters[0]) <= 2, (seed, i, infos[i].iters, ref.iters)
            if P.kappa < 1e12:
                assert abs(infos[i].iters[1] - ref.iters[1]) <= 5, (seed, i, infos[i].iters, ref.iters)


def test_batched_fallbacks_and_errors(ctx):
    """An odd leading dimension and a b that is not 16-byte aligned (the batched passes with 8-byte
    loads) beside aligned ones; problems outside the batched envelope go through fossils_solve: n > 1024,
    a rank-deficient A (truncated preconditioner) and b = 0 (x = 0); an invalid problem (m < n) gets
    its own error status while the others are solved."""
    import torch
    from paper_2406_03468_amd import binding
    good = make_problem(6000, 40, 1e6, 1e-6, seed=71)
    odd = make_problem(5000, 30, 1e4, 1e-3, seed=72)
    wide = make_problem(14000, 1030, 1e3, 1e-4, seed=73)
    rd = make_problem(4000, 25, 1e3, 1e-5, seed=74)
    rd_A = rd.A.copy()
    rd_A[:, 24] = rd_A[:, 0]  # exactly rank deficient
    zero_b = make_problem(3000, 20, 1e2, 1e-2, seed=75)
    b_off = torch.zeros(6001, dtype=torch.float64, device="cuda")
    b_off[1:] = torch.as_tensor(good.b, device="cuda")
    dev = [
        (dev_colmajor(good.A), b_off[1:]),  # b 8 bytes past a 16-byte boundary
        (dev_colmajor(odd.A, ld=5001), dev_vec(odd.b)),
        (dev_colmajor(wide.A), dev_vec(wide.b)),
        (dev_colmajor(rd_A), dev_vec(rd.b)),
        (dev_colmajor(zero_b.A), torch.zeros(3000, dtype=torch.float64, device="cuda")),
    ]
    xs = [torch.full((A.shape[1],), np.nan, dtype=torch.float64, device="cuda") for A, _ in dev]
    bad_A = torch.zeros((50, 10), dtype=torch.float64, device="cuda").t()  # 10 x 50: m < n
    bad = (bad_A, torch.zeros(10, dtype=torch.float64, device="cuda"),
           torch.zeros(50, dtype=torch.float64, device="cuda"))
    torch.cuda.synchronize()
    print("batched fallbacks", flush=True)
    s, sts, infos = binding.fossils_solve_batched(ctx, [(A, b, x) for (A, b), x in zip(dev, xs)] + [bad],
                                                  check=False)
    assert sts[5] == binding.FS_ERR_SHAPE and s == binding.FS_ERR_SHAPE, sts
    assert sts[3] == binding.FS_WARN_RANK_DEFICIENT and infos[3].rank < 25, (sts, infos[3].to_dict())
    assert np.all(host(xs[4]) == 0.0)
    for i, P in ((0, good), (1, odd)):
        ss, si, x_s = _solo(ctx, dev[i][0], dev[i][1], P.A.shape[1])
        _check_pair(P, host(xs[i]), x_s, infos[i], si, sts[i], ss, ("8-byte loads", i))
    ss, si, x_s = _solo(ctx, dev[2][0], dev[2][1], wide.A.shape[1], overlap=1)
    _check_pair(wide, host(xs[2]), x_s, infos[2], si, sts[2], ss, ("n > 1024",), same_order=False)
    # the rank-deficient one: the same truncated solve as fossils_solve
    ss, si, x_s = _solo(ctx, dev[3][0], dev[3][1], 25)
    assert ss == sts[3] and si.rank == infos[3].rank
    assert np.linalg.norm(host(xs[3]) - x_s) <= 1e-6 * np.linalg.norm(x_s)


def test_batched_large_uneven(ctx):
    """A batch of uneven larger problems (m up to 1e5, n up to 1000) with the default options."""
    import torch
    from paper_2406_03468_amd import binding
    shapes = [(100000, 400, 1e8, 1e-6), (60000, 300, 1e4, 1e-2), (24000, 1000, 1e6, 1e-8),
              (30000, 64, 1e10, 1e-10), (50001, 150, 1e3, 1.0)]
    probs = [make_problem(m, n, k, r, seed=90 + i) for i, (m, n, k, r) in enumerate(shapes)]
    dev = [(dev_colmajor(P.A), dev_vec(P.b), torch.full((P.A.shape[1],), np.nan, dtype=torch.float64, device="cuda"))
           for P in probs]
    torch.cuda.synchronize()
    print("batched large", shapes, flush=True)
    s, sts, infos = binding.fossils_solve_batched(ctx, dev)
    for i, (P, (A, b, x)) in enumerate(zip(probs, dev)):
        ss, si, xs = _solo(ctx, A, b, P.A.shape[1])
        print("checking", shapes[i], flush=True)
        _check_pair(P, host(x), xs, infos[i], si, sts[i], ss, ("large", i, shapes[i]), qr=hh.qr_lstsq_lapack)


def test_batched_edge_cases(ctx):
    """Per-problem failures stay per problem (NaN input -> FS_ERR_NONFINITE, overflowing column norms ->
    FS_ERR_TOO_LARGE, their x untouched) while the rest of the batch is solved; a square problem, a
    one-column problem with fewer rows than a pass tile, the same problem twice (the two x agree), and a
    batch of one problem."""
    import torch
    from paper_2406_03468_amd import binding
    sq = make_problem(40, 40, 1e3, 0.0, seed=81)
    one = make_problem(20, 1, 1.0, 1e-2, seed=82)
    dup = make_problem(7001, 33, 1e8, 1e-4, seed=83)
    bad = make_problem(3000, 20, 1e3, 1e-3, seed=84)
    A_nan = bad.A.copy()
    A_nan[17, 3] = np.nan
    A_big = bad.A.copy()
    A_big[:, 4] *= 1e160
    entries = [(dev_colmajor(sq.A), dev_vec(sq.b)), (dev_colmajor(one.A), dev_vec(one.b)),
               (dev_colmajor(dup.A), dev_vec(dup.b)), None, (dev_colmajor(A_nan), dev_vec(bad.b)),
               (dev_colmajor(A_big), dev_vec(bad.b))]
    entries[3] = entries[2]
    xs = [torch.full((A.shape[1],), np.nan, dtype=torch.float64, device="cuda") for A, _ in entries]
    torch.cuda.synchronize()
    print("batched edge cases", flush=True)
    s, sts, infos = binding.fossils_solve_batched(ctx, [(A, b, x) for (A, b), x in zip(entries, xs)], check=False)
    assert sts[4] == binding.FS_ERR_NONFINITE and sts[5] == binding.FS_ERR_TOO_LARGE, sts
    assert s == binding.FS_ERR_NONFINITE, s  # the first error among the problems
    assert np.all(np.isnan(host(xs[4]))) and np.all(np.isnan(host(xs[5])))
    for i, P in ((0, sq), (1, one), (2, dup), (3, dup)):
        ss, si, x_s = _solo(ctx, entries[i][0], entries[i][1], P.A.shape[1])
        assert sts[i] == ss, (i, sts, ss)
        xb = host(xs[i])
        assert np.all(np.isfinite(xb)), i
        assert be.relative_backward_error(P.A, P.b, xb, P.sigma, P.V) <= 1e-14, i
        ref = max(np.linalg.norm(hh.qr_lstsq(P.A, P.b) - P.x_true) / np.linalg.norm(P.x_true), P.kappa * U)
        assert np.linalg.norm(xb - x_s) / np.linalg.norm(P.x_true) <= 10 * ref, (i, ref)
    ref_dup = max(np.linalg.norm(hh.qr_lstsq(dup.A, dup.b) - dup.x_true) / np.linalg.norm(dup.x_true), dup.kappa * U)
    assert np.linalg.norm(host(xs[2]) - host(xs[3])) / np.linalg.norm(dup.x_true) <= 10 * ref_dup
    # a batch of one
    x1 = torch.full((33,), np.nan, dtype=torch.float64, device="cuda")
    s1, sts1, inf1 = binding.fossils_solve_batched(ctx, [(entries[2][0], entries[2][1], x1)])
    assert s1 == sts1[0] == sts[2] and inf1[0].iters[0] > 0
    assert np.linalg.norm(host(x1) - host(xs[2])) / np.linalg.norm(dup.x_true) <= 10 * ref_dup
