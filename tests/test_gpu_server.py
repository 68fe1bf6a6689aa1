"""Serving runtime on the GPU: a mixed stream of independent requests drained by worker slots
(continuous batching).  Every request must meet the single-solve bar (BE <= 1e-14, forward error
within 10x of Householder QR's) whether it runs alone or inside the mix."""

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


def _mix(seed=11, count=24):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(rng.integers(20, 200))
        m = int(rng.integers(max(20 * n, 2000), 30000))
        kappa = 10.0 ** rng.uniform(2, 12)
        rn = 10.0 ** rng.uniform(-12, 0)
        out.append((make_problem(m, n, kappa, rn, seed=100 + i), int(rng.integers(0, 2))))
    return out


def test_mixed_stream_all_backward_stable(ctx):
    import torch
    from paper_2406_03468_amd import binding
    srv = binding.Server(ctx, hbm_budget=8 << 30, max_slots=4)
    try:
        probs = _mix()
        dev = [(dev_colmajor(P.A), dev_vec(P.b), torch.zeros(P.A.shape[1], dtype=torch.float64, device="cuda"))
               for P, _ in probs]
        torch.cuda.synchronize()
        # every other pair of requests runs the mixed-precision form (FP32 sketch, FP64 fallback)
        om = [None] * len(probs)
        for i, (P, _) in enumerate(probs):
            if (i // 2) % 2:
                om[i] = binding.fs_options_default(*P.A.shape)
                om[i].precision = binding.FS_MIXED
        tickets = [binding.batched_submit(srv, A, b, x, method=meth, opts=o)
                   for (A, b, x), (_, meth), o in zip(dev, probs, om)]
        for t in tickets:
            binding.fs_server_wait(srv, t)
        for t, (P, meth), (_, _, x), o in zip(tickets, probs, dev, om):
            done, status, info = binding.batched_poll(srv, t)
            assert done and status in (0, binding.FS_WARN_NOT_CONVERGED), (status, info.to_dict())
            fb = bool(info.flags & binding.FS_FLAG_FP64_SKETCH)
            # the fallback is taken exactly when the FP32 sketch's condest passes u32 condest > 2
            # (info.condest is then the FP64 sketch's, equal to it up to u32 condest relative)
            if o is None:
                assert not fb
            else:
                assert (info.condest * 2.0**-24 > 1.6) if fb else (info.condest * 2.0**-24 <= 2.0), info.to_dict()
            xh = host(x)
            bg = be.relative_backward_error(P.A, P.b, xh, P.sigma, P.V)
            assert bg <= 1e-14, (P.A.shape, P.kappa, meth, bg, info.to_dict())
            xq = hh.qr_lstsq(P.A, P.b)
            fe = np.linalg.norm(xh - P.x_true) / np.linalg.norm(P.x_true)
            fq = max(np.linalg.norm(xq - P.x_true) / np.linalg.norm(P.x_true), P.kappa * U)
            assert fe <= 10 * fq
            ts, tst, tf = binding.fs_server_ticket_times(srv, t)
            assert 0 <= ts <= tst <= tf
    finally:
        srv.close()


def test_solo_vs_mix(ctx):
    """A request solved alone (fossils_solve on its own context) and inside the mixed stream gives
    the same quality and the same iteration counts up to the rounding of the sketch sums."""
    import torch
    from paper_2406_03468_amd import binding
    P = make_problem(12000, 150, 1e10, 1e-6, seed=77)
    A, b = dev_colmajor(P.A), dev_vec(P.b)
    x_solo = torch.zeros(150, dtype=torch.float64, device="cuda")
    _, info_solo = binding.fossils_solve(ctx, A, b, x_solo)
    srv = binding.Server(ctx, hbm_budget=8 << 30, max_slots=3)
    try:
        others = _mix(seed=5, count=8)
        keep = [(dev_colmajor(Q.A), dev_vec(Q.b), torch.zeros(Q.A.shape[1], dtype=torch.float64, device="cuda"))
                for Q, _ in others]
        x_mix = torch.zeros(150, dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        ts = [binding.batched_submit(srv, a, bb, xx) for a, bb, xx in keep[:4]]
        t = binding.batched_submit(srv, A, b, x_mix)
        ts += [binding.batched_submit(srv, a, bb, xx) for a, bb, xx in keep[4:]]
        for tt in ts + [t]:
            binding.fs_server_wait(srv, tt)
        _, status, info_mix = binding.batched_poll(srv, t)
    finally:
        srv.close()
    b_solo = be.relative_backward_error(P.A, P.b, host(x_solo), P.sigma, P.V)
    b_mix = be.relative_backward_error(P.A, P.b, host(x_mix), P.sigma, P.V)
    assert b_solo <= 1e-14 and b_mix <= 1e-14
    assert abs(info_mix.iters[0] - info_solo.iters[0]) <= 2 and abs(info_mix.iters[1] - info_solo.iters[1]) <= 5
    assert abs(info_mix.condest - info_solo.condest) <= 1e-6 * info_solo.condest


def test_admission_and_tickets(ctx):
    import torch
    from paper_2406_03468_amd import binding
    P = make_problem(20000, 100, 1e4, 1e-3, seed=3)
    A, b = dev_colmajor(P.A), dev_vec(P.b)
    x = torch.zeros(100, dtype=torch.float64, device="cuda")
    need = binding.fs_solve_footprint(20000, 100)
    srv = binding.Server(ctx, hbm_budget=2 * (need // 2), max_slots=2)  # share per slot < need
    try:
        with pytest.raises(binding.FossilsError) as e:
            binding.batched_submit(srv, A, b, x)
        assert e.value.status == binding.FS_ERR_TOO_LARGE
        with pytest.raises(binding.FossilsError) as e:
            binding.batched_poll(srv, 12345)
        assert e.value.status == binding.FS_ERR_UNKNOWN_TICKET
    finally:
        srv.close()
