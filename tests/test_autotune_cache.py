"""Host logic of the fused-pass tuning cache (no GPU): keys, file round trip, loading filtered by
architecture and dtype, and the ABI's refusal of a null context before any device work."""

import ctypes

from paper_2406_03468_amd import autotune, binding


def test_m_bucket_is_floor_log2():
    assert [autotune.m_bucket(m) for m in (1, 2, 3, 4, 1023, 1024, 1_000_000)] == [0, 1, 1, 2, 9, 10, 19]
    assert autotune.key("gfx950", 1000, 1_000_000) == "gfx950|1000|19|f64"


def test_cache_round_trip_and_apply(tmp_path):
    p = str(tmp_path / "tune.json")
    assert autotune.load(p) == {}
    cache = {autotune.key("gfx950", 1000, 1_000_000): {"H": 16, "G": 256, "ms": 1.3},
             autotune.key("gfx950", 200, 20000): {"H": 32, "G": 128, "ms": 0.05},
             autotune.key("gfx942", 1000, 1_000_000): {"H": 8, "G": 304, "ms": 1.9},
             "gfx950|1000|19|f32": {"H": 16, "G": 256, "ms": 0.7}}
    autotune.save(cache, p)
    assert autotune.load(p) == cache
    got = []
    n = autotune.apply("ctx", autotune.load(p), arch="gfx950", set_fn=lambda *a: got.append(a))
    assert n == 2
    assert sorted(got) == sorted([("ctx", 1 << 19, 1000, 16, 256), ("ctx", 1 << 14, 200, 32, 128)])


def test_tuning_calls_refuse_a_null_context():
    lib = binding.load()
    c = ctypes.c_void_p
    assert lib.fs_set_pass_tuning(None, 1000, 100, 16, 256) == binding.FS_ERR_INVALID_ARG
    assert lib.fs_clear_pass_tuning(None) == binding.FS_ERR_INVALID_ARG
    assert lib.fs_tune_pass(None, 1000, 100, c(8), 1000, c(8), c(8), 3, None, None, None) == binding.FS_ERR_INVALID_ARG
