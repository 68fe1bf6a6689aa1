"""The fused-pass autotuner on the GPU (fs_tune_pass / fs_set_pass_tuning through the C ABI): the
kept (tile height, work-group count) is admissible; the pass it gives matches the built-in one to
the rounding of the partial sums and is then used by every pass of that shape (bit-identical
repeats); a solve with it meets the bar with the same iteration counts; inadmissible pairs are
refused; the JSON cache reloads the same configuration."""

import numpy as np
import pytest

from gpu_util import dev_colmajor, dev_vec, host
from oracle import backward_error as be
from synth import make_problem

pytestmark = pytest.mark.gpu


def _admissible(H, n):
    L = -(-n * H // 1024)
    # 32-row tiles up to 32 column slots (the residual pass runs those above 8 with 16-row tiles)
    return {64: 1 <= L <= 4, 32: 1 <= L <= 32, 16: 1 <= L <= 16, 8: 5 <= L <= 16, 4: 5 <= L <= 16}.get(H, False)


@pytest.mark.parametrize("m,n", [(200000, 500), (30001, 1000), (5003, 60)])
def test_tuned_pass(m, n):
    import torch
    from paper_2406_03468_amd import autotune, binding
    ctx = binding.Context(0)
    try:
        rng = np.random.default_rng(m + n)
        A = dev_colmajor(rng.standard_normal((m, n)), ld=m + 3)
        z = dev_vec(rng.standard_normal(n))
        v0 = torch.empty(n, dtype=torch.float64, device="cuda")
        binding.fs_normal_pass(ctx, A, z, v0)
        v1 = torch.empty_like(v0)
        H, G, ms = binding.fs_tune_pass(ctx, A, z, v1, repeats=3)
        nc = torch.cuda.get_device_properties(0).multi_processor_count
        assert _admissible(H, n) and G % 8 == 0 and 8 <= G <= 2 * nc and ms > 0, (H, G, ms)
        assert torch.linalg.norm(v1 - v0) <= 1e-13 * torch.linalg.norm(v0)
        v2 = torch.empty_like(v0)
        binding.fs_normal_pass(ctx, A, z, v2)  # the kept pair, same fixed-order sums
        assert torch.equal(v2, v1)
        bad_H = 64 if not _admissible(64, n) else 4
        with pytest.raises(binding.FossilsError):
            binding.fs_set_pass_tuning(ctx, m, n, bad_H, 256)
        with pytest.raises(binding.FossilsError):
            binding.fs_set_pass_tuning(ctx, m, n, H, 100)
        # the cache: record, clear, reload
        cache = {}
        autotune.tune(ctx, A, z, v1, cache=cache, repeats=2)
        Hc, Gc = cache[autotune.key(autotune.device_arch(), n, m)]["H"], cache[autotune.key(autotune.device_arch(), n, m)]["G"]
        binding.fs_clear_pass_tuning(ctx)
        assert autotune.apply(ctx, cache) == 1
        v3 = torch.empty_like(v0)
        binding.fs_normal_pass(ctx, A, z, v3)
        binding.fs_clear_pass_tuning(ctx)
        binding.fs_set_pass_tuning(ctx, m, n, Hc, Gc)
        v4 = torch.empty_like(v0)
        binding.fs_normal_pass(ctx, A, z, v4)
        assert torch.equal(v3, v4)
    finally:
        ctx.close()


def test_solve_with_a_tuned_pass():
    import torch
    from paper_2406_03468_amd import binding
    P = make_problem(100000, 300, 1e8, 1e-6, seed=21)
    ctx = binding.Context(0)
    try:
        A, b = dev_colmajor(P.A), dev_vec(P.b)
        res = []
        for tuned in (False, True):
            if tuned:
                z = dev_vec(np.ones(300))
                v = torch.empty(300, dtype=torch.float64, device="cuda")
                binding.fs_tune_pass(ctx, A, z, v, repeats=2)
            x = torch.zeros(300, dtype=torch.float64, device="cuda")
            st, info = binding.fossils_solve(ctx, A, b, x)
            assert st == 0, info.to_dict()
            assert be.relative_backward_error(P.A, P.b, host(x), P.sigma, P.V) <= 1e-14
            res.append(list(info.iters))
        assert abs(res[0][0] - res[1][0]) <= 1 and abs(res[0][1] - res[1][1]) <= 5, res
    finally:
        ctx.close()
