"""The library's host code built with AddressSanitizer and UndefinedBehaviorSanitizer (device code
unchanged; the sanitizers apply to the host pass only), linked into a C driver that exercises the
C ABI's validation paths, options, footprints and status strings without a GPU.  Any invalid host
memory access or undefined behaviour fails the test."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-g"]

pytestmark = pytest.mark.slow


def _hipcc():
    for c in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if c and os.path.exists(c):
            return c
    pytest.skip("hipcc not available")


def test_abi_validation_under_asan_ubsan(tmp_path):
    import concurrent.futures as cf

    from paper_2406_03468_amd import build as b
    hipcc = _hipcc()
    flags = [f for f in b.HIPFLAGS if f != "-O3"] + ["-O1"] + SAN

    def compile_one(src):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        r = subprocess.run([hipcc, *flags, "-c", src, "-o", obj], capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-3000:]
        return obj

    with cf.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(compile_one, b.sources()))
    lib = str(tmp_path / "libfossils_san.so")
    r = subprocess.run([hipcc, "-shared", "-fPIC", f"--offload-arch={b.ARCH}", *SAN, "-o", lib, *objs],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    exe = str(tmp_path / "sanitize_driver")
    r = subprocess.run([hipcc, "-x", "c", "-O1", "-g", *SAN[:4], "-I", os.path.join(ROOT, "include"),
                        os.path.join(ROOT, "tests", "sanitize_driver.c"), "-x", "none", lib, "-o", exe,
                        f"-Wl,-rpath,{tmp_path}"], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0 and "sanitized host checks passed" in r.stdout, (r.stdout[-2000:], r.stderr[-4000:])
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
