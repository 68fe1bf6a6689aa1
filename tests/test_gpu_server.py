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


def _opts(P, mixed):
    """The options a multi-slot server runs a request with (overlap_svd off), FP64 or mixed."""
    from paper_2406_03468_amd import binding
    o = binding.fs_options_default(*P.A.shape)
    o.overlap_svd = 0
    if mixed:
        o.precision = binding.FS_MIXED
    return o


def test_solo_vs_mix(ctx):
    """Every request of a mixed stream (FOSSILS and SPIR, FP64 and mixed precision) gives the same x
    alone (the plain solver on the caller's context, with the options the server runs it with) and
    inside the mix (4 slots sharing the GPU): both meet the bar, and the two solutions agree to the
    forward-error scale (10x Householder QR's, floored at kappa u).  They are not bitwise equal: the
    sketch's sums are accumulated with device atomics in a run-dependent order."""
    import torch
    from paper_2406_03468_amd import binding
    probs = _mix(seed=5, count=12)
    dev = [(dev_colmajor(P.A), dev_vec(P.b)) for P, _ in probs]
    opts = [_opts(P, (i // 2) % 2 == 1) for i, (P, _) in enumerate(probs)]
    solo, solo_info = [], []
    for (A, b), (P, meth), o in zip(dev, probs, opts):
        x = torch.zeros(P.A.shape[1], dtype=torch.float64, device="cuda")
        fn = binding.spir_solve if meth == 1 else binding.fossils_solve
        st, info = fn(ctx, A, b, x, o)
        assert st in (0, binding.FS_WARN_NOT_CONVERGED), info.to_dict()
        solo.append(host(x))
        solo_info.append(info)
    xs_mix = [torch.zeros(P.A.shape[1], dtype=torch.float64, device="cuda") for P, _ in probs]
    srv = binding.Server(ctx, hbm_budget=8 << 30, max_slots=4)
    try:
        tickets = [binding.batched_submit(srv, A, b, x, method=meth, opts=o)
                   for (A, b), (_, meth), o, x in zip(dev, probs, opts, xs_mix)]
        for t in tickets:
            binding.fs_server_wait(srv, t)
        mix_info = [binding.batched_poll(srv, t)[2] for t in tickets]
        # the requests overlapped on the device
        times = [binding.fs_server_ticket_times(srv, t) for t in tickets]
        assert any(times[i][1] < times[j][2] and times[j][1] < times[i][2]
                   for i in range(len(times)) for j in range(i + 1, len(times)))
    finally:
        srv.close()
    for i, (P, meth) in enumerate(probs):
        x_mix, x_solo = host(xs_mix[i]), solo[i]
        b_solo = be.relative_backward_error(P.A, P.b, x_solo, P.sigma, P.V)
        b_mix = be.relative_backward_error(P.A, P.b, x_mix, P.sigma, P.V)
        assert b_solo <= 1e-14 and b_mix <= 1e-14, (i, b_solo, b_mix)
        xq = hh.qr_lstsq(P.A, P.b)
        ref = max(np.linalg.norm(v - P.x_true) / np.linalg.norm(P.x_true) for v in (xq, x_solo))
        ref = max(ref, P.kappa * U)
        assert np.linalg.norm(x_mix - x_solo) / np.linalg.norm(P.x_true) <= 10 * ref, (i, P.kappa, ref)
        fm, fs = mix_info[i].flags & binding.FS_FLAG_FP64_SKETCH, solo_info[i].flags & binding.FS_FLAG_FP64_SKETCH
        if abs(np.log2(max(solo_info[i].condest, 1.0) * 2.0**-24)) > 0.5:  # away from the mixed threshold
            assert fm == fs, (i, mix_info[i].to_dict(), solo_info[i].to_dict())
        # condest moves with the rounding of the sketch's atomic sums: |d sigma_min| <~ u ||S A||_F
        cs = solo_info[i].condest
        assert abs(mix_info[i].condest - cs) <= 50 * U * np.sqrt(P.A.shape[1]) * cs**2 + 1e-10 * cs
        assert abs(mix_info[i].iters[0] - solo_info[i].iters[0]) <= 2, (i, mix_info[i].iters, solo_info[i].iters)
        if P.kappa < 1e12:
            assert abs(mix_info[i].iters[1] - solo_info[i].iters[1]) <= 5, (i, mix_info[i].iters, solo_info[i].iters)


def test_admission_and_tickets(ctx):
    import torch
    from paper_2406_03468_amd import binding
    P = make_problem(20000, 100, 1e4, 1e-3, seed=3)
    A, b = dev_colmajor(P.A), dev_vec(P.b)
    x = torch.zeros(100, dtype=torch.float64, device="cuda")
    probe = binding.Server(ctx, hbm_budget=1 << 40, max_slots=2)
    need = binding.fs_server_request_footprint(probe, 20000, 100)
    probe.close()
    srv = binding.Server(ctx, hbm_budget=need - 1, max_slots=2)  # the whole ledger is too small
    try:
        with pytest.raises(binding.FossilsError) as e:
            binding.batched_submit(srv, A, b, x)
        assert e.value.status == binding.FS_ERR_TOO_LARGE
        with pytest.raises(binding.FossilsError) as e:
            binding.batched_poll(srv, 12345)
        assert e.value.status == binding.FS_ERR_UNKNOWN_TICKET
    finally:
        srv.close()
    srv = binding.Server(ctx, hbm_budget=need, max_slots=2)  # exactly one request's footprint: admitted
    try:
        t = binding.batched_submit(srv, A, b, x)
        binding.fs_server_wait(srv, t)
        assert binding.batched_poll(srv, t)[1] == 0
        used, peak, budget = binding.fs_server_memory(srv)
        assert peak <= budget == need and used <= budget
    finally:
        srv.close()
    assert be.relative_backward_error(P.A, P.b, host(x), P.sigma, P.V) <= 1e-14


def test_ledger_admits_as_memory_frees(ctx):
    """A ledger that holds one large request at a time (1.5 footprints) and 3 slots: large and small
    requests are all admitted (none refused), the charge never exceeds the budget, no two large
    requests run at once, and a small request runs beside a large one when it fits."""
    import torch
    from paper_2406_03468_amd import binding
    big = [make_problem(60000, 400, 1e8, 1e-6, seed=40 + i) for i in range(3)]
    small = [make_problem(4000, 30, 1e6, 1e-4, seed=50 + i) for i in range(3)]
    probe = binding.Server(ctx, hbm_budget=1 << 40, max_slots=3)
    fb = binding.fs_server_request_footprint(probe, 60000, 400)
    fsm = binding.fs_server_request_footprint(probe, 4000, 30)
    probe.close()
    assert 2 * fsm < fb // 2
    budget = fb + fb // 2
    order = [big[0], small[0], big[1], small[1], big[2], small[2]]
    dev = [(dev_colmajor(P.A), dev_vec(P.b), torch.zeros(P.A.shape[1], dtype=torch.float64, device="cuda"))
           for P in order]
    srv = binding.Server(ctx, hbm_budget=budget, max_slots=3)
    try:
        tickets = [binding.batched_submit(srv, A, b, x) for A, b, x in dev]
        for t in tickets:
            binding.fs_server_wait(srv, t)
        res = [binding.batched_poll(srv, t) for t in tickets]
        times = [binding.fs_server_ticket_times(srv, t) for t in tickets]
        used, peak, bud = binding.fs_server_memory(srv)
    finally:
        srv.close()
    assert all(r[0] and r[1] == 0 for r in res), [r[1] for r in res]
    assert peak <= bud == budget and used <= budget, (used, peak, budget)
    bigs = [times[i] for i in (0, 2, 4)]
    for i in range(3):
        for j in range(i + 1, 3):
            assert bigs[i][2] <= bigs[j][1] or bigs[j][2] <= bigs[i][1], bigs  # never two at once
    for P, (_, _, x) in zip(order, dev):
        assert be.relative_backward_error(P.A, P.b, host(x), P.sigma, P.V) <= 1e-14


def test_submit_waits_for_the_callers_stream(ctx):
    """A and b are produced on a side stream that is still busy at submission (a long device sleep
    ahead of the copies): the solve starts after them and sees the finished inputs."""
    import torch
    from paper_2406_03468_amd import binding
    P = make_problem(30000, 120, 1e6, 1e-5, seed=61)
    src_A, src_b = dev_colmajor(P.A), dev_vec(P.b)
    A = torch.full((120, 30000), float("nan"), dtype=torch.float64, device="cuda").t()
    b = torch.full((30000,), float("nan"), dtype=torch.float64, device="cuda")
    x = torch.zeros(120, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    srv = binding.Server(ctx, hbm_budget=4 << 30, max_slots=2)
    try:
        with torch.cuda.stream(side):
            torch.cuda._sleep(200_000_000)  # ~0.1 s of device time before the inputs exist
            A.copy_(src_A)
            b.copy_(src_b)
            t = binding.batched_submit(srv, A, b, x)  # orders after `side` (torch's current stream here)
        binding.fs_server_wait(srv, t)
        _, status, info = binding.batched_poll(srv, t)
    finally:
        srv.close()
    assert status == 0, (status, info.to_dict() if info else None)
    assert be.relative_backward_error(P.A, P.b, host(x), P.sigma, P.V) <= 1e-14
