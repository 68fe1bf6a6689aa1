"""C ABI checks that need no GPU: the library loads, exports every declared symbol, and rejects
bad arguments before touching a device."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fossils.h")


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*([A-Za-z_][A-Za-z0-9_]*)\s*\(", txt, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "return")))


@pytest.fixture(scope="module")
def clib():
    from paper_2406_03468_amd import binding
    return binding.load()


def test_header_parses():
    names = declared_functions()
    for must in ("fossils_solve", "spir_solve", "sketch_create", "sketch_apply", "fs_normal_pass"):
        assert must in names


def test_library_exports_every_declared_symbol(clib):
    for name in declared_functions():
        assert hasattr(clib, name), name


def test_binding_names_match_header():
    from paper_2406_03468_amd import binding
    assert sorted(binding.exported_names()) == declared_functions()


def test_options_default_is_algorithm4(clib):
    from paper_2406_03468_amd import binding
    o = binding.fs_options_default(1_000_000, 1000)
    assert (o.d, o.zeta, o.kw_every, o.max_inner) == (12000, 8, 5, 100)
    assert (o.gamma, o.rho, o.tau_factor) == (10.0, 0.4, 30.0)
    assert o.column_scaling == 1 and o.steps == 2 and o.fixed_q == 0
    assert o.precond == binding.FS_PRECOND_SVD  # Alg 4: P = V Sigma^{-1}
    # the last fields: the ctypes layout agrees with the header's
    assert (o.overlap_svd, o.graph_sweeps, o.overlap_pass_groups) == (1, 0, 0)


def test_status_strings(clib):
    assert clib.fs_status_string(0) == b"FS_OK"
    assert clib.fs_status_string(-2) == b"FS_ERR_SHAPE"
    assert clib.fs_status_string(1) == b"FS_WARN_RANK_DEFICIENT"


def test_validation_before_device_work(clib):
    from paper_2406_03468_amd import binding
    o = binding.FsOptions()
    # null context
    assert clib.fossils_solve(None, 10, 2, None, 10, None, None, None, None) == binding.FS_ERR_INVALID_ARG
    assert clib.spir_solve(None, 10, 2, None, 10, None, None, None, None) == binding.FS_ERR_INVALID_ARG
    # shape errors in options defaulting
    assert clib.fs_options_default(5, 10, ctypes.byref(o)) == binding.FS_ERR_SHAPE
    assert clib.fs_options_default(5, 0, ctypes.byref(o)) == binding.FS_ERR_SHAPE
    assert clib.fs_options_default(5, 2, None) == binding.FS_ERR_INVALID_ARG
    assert clib.sketch_create(None, 10, 5, 2, 1, None) == binding.FS_ERR_INVALID_ARG
    assert clib.fs_sketch_qr(None, 10, 2, None, 10) == binding.FS_ERR_INVALID_ARG
    assert clib.fs_triangular_inverse(None, 2, None, 2, None) == binding.FS_ERR_INVALID_ARG
    # the batched and no-allocation entry points validate before any device work
    probs = (binding.FsProblem * 1)()
    sts = (ctypes.c_int32 * 1)()
    assert clib.fossils_solve_batched(None, 1, probs, None, None, sts) == binding.FS_ERR_INVALID_ARG
    assert clib.fossils_solve_batched(None, 0, probs, None, None, sts) == binding.FS_ERR_INVALID_ARG
    assert clib.fossils_solve_noalloc(None, 10, 2, None, 10, None, None, None, None) == binding.FS_ERR_INVALID_ARG


def test_problem_struct_layout():
    """fs_problem's ctypes layout matches the header's C layout (offsets of every field)."""
    from paper_2406_03468_amd import binding
    offs = {name: getattr(binding.FsProblem, name).offset for name, _ in binding.FsProblem._fields_}
    assert offs == {"m": 0, "n": 8, "A": 16, "lda": 24, "b": 32, "x": 40, "method": 48}
    assert ctypes.sizeof(binding.FsProblem) == 56


def test_missing_library_fails_loudly(tmp_path):
    from paper_2406_03468_amd import binding
    with pytest.raises(FileNotFoundError):
        binding.load(str(tmp_path / "nope.so"))


def test_solve_footprint_and_server_validation(clib):
    """Workspace footprint used for serving admission: positive, growing with m and n; invalid
    shapes give 0.  Server creation validates its arguments before touching the device."""
    from paper_2406_03468_amd import binding
    f1 = binding.fs_solve_footprint(100_000, 100)
    f2 = binding.fs_solve_footprint(200_000, 100)
    f3 = binding.fs_solve_footprint(100_000, 200)
    assert 0 < f1 < f2 and f1 < f3
    # the index stream (m zeta 2 bytes) and the sketch (12 n x (n+1) doubles) are both counted
    assert f1 >= 100_000 * 8 * 2 + 8 * 1200 * 101
    assert binding.fs_solve_footprint(10, 20) == 0
    h = ctypes.c_void_p()
    assert clib.fs_server_create(None, 1 << 30, 2, ctypes.byref(h)) == binding.FS_ERR_INVALID_ARG
    assert clib.batched_submit(None, None, None) == binding.FS_ERR_INVALID_ARG
