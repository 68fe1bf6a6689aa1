"""Thin ctypes binding of libfossils.so (argument marshalling only).

Every function mirrors the C entry point of the same name in include/fossils.h.  Tensors are torch
tensors in device memory; torch provides memory and the current HIP stream, nothing else.  Matrices
are column-major: a torch (rows, cols) tensor with strides (1, ld), e.g. ``M.t().contiguous().t()``.
There is no fallback: if the library is missing, ``load()`` raises.
"""

from __future__ import annotations

import ctypes
import os
import sys
from typing import Optional

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "libfossils.so")

FS_OK = 0
FS_WARN_RANK_DEFICIENT = 1
FS_WARN_NOT_CONVERGED = 2
FS_ERR_INVALID_ARG = -1
FS_ERR_SHAPE = -2
FS_ERR_NOMEM = -3
FS_ERR_DEVICE = -4
FS_ERR_NONFINITE = -5
FS_ERR_TOO_LARGE = -6
FS_ERR_UNKNOWN_TICKET = -7
FS_ERR_UNSUPPORTED = -8

FS_PRECOND_QR = 0
FS_PRECOND_SVD = 1
FS_FP64 = 0
FS_MIXED = 1
FS_INIT_SKETCH = 0
FS_INIT_ZERO = 1
FS_FLAG_RANK_DEFICIENT = 1
FS_FLAG_NOT_CONVERGED = 2
FS_FLAG_FP64_SKETCH = 4
FS_FLAG_EARLY_SECOND_STEP = 8
FS_FLAG_SVD_ABANDONED = 16

c_int32, c_int64, c_uint64, c_double, c_vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double, ctypes.c_void_p


class FsOptions(ctypes.Structure):
    _fields_ = [
        ("d", c_int32), ("zeta", c_int32), ("seed", c_uint64), ("eta", c_double), ("eta_factor", c_double),
        ("gamma", c_double), ("rho", c_double), ("kw_every", c_int32), ("max_inner", c_int32),
        ("tau_factor", c_double), ("column_scaling", c_int32), ("precond", c_int32), ("fixed_q", c_int32),
        ("steps", c_int32), ("precision", c_int32), ("max_sweeps", c_int32), ("init", c_int32),
        ("overlap_svd", c_int32), ("graph_sweeps", c_int32), ("overlap_pass_groups", c_int32),
    ]


class FsInfo(ctypes.Structure):
    _fields_ = [
        ("iters", c_int32 * 2), ("flags", c_int32), ("rank", c_int32), ("be_sk", c_double),
        ("normest", c_double), ("condest", c_double), ("cnorm", c_double * 2), ("svd_sweeps", c_int32),
        ("kw_evals", c_int32), ("phase_ms", c_double * 6),
    ]

    def to_dict(self):
        return {
            "iters": [self.iters[0], self.iters[1]], "flags": self.flags, "rank": self.rank,
            "be_sk": self.be_sk, "normest": self.normest, "condest": self.condest,
            "cnorm": [self.cnorm[0], self.cnorm[1]], "svd_sweeps": self.svd_sweeps,
            "kw_evals": self.kw_evals, "phase_ms": list(self.phase_ms),
        }


class FsProblem(ctypes.Structure):
    _fields_ = [("m", c_int64), ("n", c_int32), ("A", c_vp), ("lda", c_int64), ("b", c_vp), ("x", c_vp),
                ("method", c_int32)]


class FsRequest(ctypes.Structure):
    _fields_ = [("method", c_int32), ("m", c_int64), ("n", c_int32), ("A", c_vp), ("lda", c_int64), ("b", c_vp),
                ("x", c_vp), ("opts", ctypes.POINTER(FsOptions)), ("stream", c_vp)]


FS_METHOD_FOSSILS = 0
FS_METHOD_SPIR = 1
FS_METHOD_SPIR_LSQR = 2


class FossilsError(RuntimeError):
    def __init__(self, status, detail=""):
        self.status = status
        super().__init__(f"{status_string(status)} {detail}".strip())


_lib = None

# (name, restype, argtypes)
_SIGS = [
    ("fs_status_string", ctypes.c_char_p, [c_int32]),
    ("fs_last_error_detail", ctypes.c_char_p, []),
    ("fs_context_create", c_int32, [ctypes.c_int, c_vp, ctypes.POINTER(c_vp)]),
    ("fs_context_destroy", c_int32, [c_vp]),
    ("fs_options_default", c_int32, [c_int64, c_int32, ctypes.POINTER(FsOptions)]),
    ("fossils_solve", c_int32, [c_vp, c_int64, c_int32, c_vp, c_int64, c_vp, c_vp, ctypes.POINTER(FsOptions),
                                ctypes.POINTER(FsInfo)]),
    ("spir_solve", c_int32, [c_vp, c_int64, c_int32, c_vp, c_int64, c_vp, c_vp, ctypes.POINTER(FsOptions),
                             ctypes.POINTER(FsInfo)]),
    ("spir_lsqr_solve", c_int32, [c_vp, c_int64, c_int32, c_vp, c_int64, c_vp, c_vp, ctypes.POINTER(FsOptions),
                                  ctypes.POINTER(FsInfo)]),
    ("fossils_solve_complex", c_int32, [c_vp, c_int64, c_int32, c_vp, c_int64, c_vp, c_vp, ctypes.POINTER(FsOptions),
                                        ctypes.POINTER(FsInfo)]),
    ("spir_solve_complex", c_int32, [c_vp, c_int64, c_int32, c_vp, c_int64, c_vp, c_vp, ctypes.POINTER(FsOptions),
                                     ctypes.POINTER(FsInfo)]),
    ("fossils_solve_multi", c_int32, [c_vp, c_int64, c_int32, c_vp, c_int64, c_int32, c_vp, c_int64, c_vp, c_int64,
                                      ctypes.POINTER(FsOptions), ctypes.POINTER(FsInfo)]),
    ("fossils_solve_batched", c_int32, [c_vp, c_int32, ctypes.POINTER(FsProblem), ctypes.POINTER(FsOptions),
                                        ctypes.POINTER(FsInfo), ctypes.POINTER(c_int32)]),
    ("fossils_solve_noalloc", c_int32, [c_vp, c_int64, c_int32, c_vp, c_int64, c_vp, c_vp, ctypes.POINTER(FsOptions),
                                        ctypes.POINTER(FsInfo)]),
    ("fossils_solve_mixed", c_int32, [c_vp, c_int64, c_int32, c_vp, c_int64, c_vp, c_int64, c_vp, c_vp,
                                      ctypes.POINTER(FsOptions), ctypes.POINTER(FsInfo)]),
    ("fs_to_fp32", c_int32, [c_vp, c_int64, c_int32, c_vp, c_int64, c_vp, c_int64]),
    ("fs_server_create", c_int32, [c_vp, ctypes.c_size_t, c_int32, ctypes.POINTER(c_vp)]),
    ("fs_server_destroy", c_int32, [c_vp]),
    ("batched_submit", c_int32, [c_vp, ctypes.POINTER(FsRequest), ctypes.POINTER(c_uint64)]),
    ("batched_poll", c_int32, [c_vp, c_uint64, ctypes.POINTER(c_int32), ctypes.POINTER(c_int32),
                               ctypes.POINTER(FsInfo)]),
    ("fs_server_wait", c_int32, [c_vp, c_uint64]),
    ("fs_server_ticket_times", c_int32, [c_vp, c_uint64, ctypes.POINTER(c_double), ctypes.POINTER(c_double),
                                         ctypes.POINTER(c_double)]),
    ("fs_solve_footprint", ctypes.c_size_t, [c_int64, c_int32, ctypes.POINTER(FsOptions)]),
    ("fs_server_memory", c_int32, [c_vp, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t),
                                   ctypes.POINTER(ctypes.c_size_t)]),
    ("fs_server_request_footprint", c_int32, [c_vp, c_int64, c_int32, ctypes.POINTER(FsOptions),
                                              ctypes.POINTER(ctypes.c_size_t)]),
    ("fs_context_workspace", c_int32, [c_vp, ctypes.POINTER(ctypes.c_size_t)]),
    ("fs_context_trim", c_int32, [c_vp]),
    ("sketch_create", c_int32, [c_vp, c_int64, c_int32, c_int32, c_uint64, ctypes.POINTER(c_vp)]),
    ("sketch_destroy", c_int32, [c_vp]),
    ("sketch_indices", c_int32, [c_vp, c_int64, c_int64, c_vp, c_vp]),
    ("sketch_apply", c_int32, [c_vp, c_int32, c_vp, c_int64, c_vp, c_vp, c_int64, c_vp, c_int32]),
    ("fs_sketch_qr", c_int32, [c_vp, c_int32, c_int32, c_vp, c_int64]),
    ("fs_svd_triangular", c_int32, [c_vp, c_int32, c_vp, c_int64, c_vp, c_vp, c_int64, ctypes.POINTER(c_int32)]),
    ("fs_normal_pass", c_int32, [c_vp, c_int64, c_int32, c_vp, c_int64, c_vp, c_vp]),
    ("fs_residual_pass", c_int32, [c_vp, c_int64, c_int32, c_vp, c_int64, c_vp, c_vp, c_vp,
                                   ctypes.POINTER(c_double)]),
    ("fs_trsv", c_int32, [c_vp, c_int32, c_vp, c_int64, c_int32, c_vp, c_vp]),
    ("fs_triangular_inverse", c_int32, [c_vp, c_int32, c_vp, c_int64, c_vp]),
    ("fs_time_normal_pass", c_int32, [c_vp, c_int64, c_int32, c_vp, c_int64, c_vp, c_vp, c_int32,
                                      ctypes.POINTER(c_double), ctypes.POINTER(c_double)]),
    ("fs_tune_pass", c_int32, [c_vp, c_int64, c_int32, c_vp, c_int64, c_vp, c_vp, c_int32,
                               ctypes.POINTER(c_int32), ctypes.POINTER(c_int32), ctypes.POINTER(c_double)]),
    ("fs_set_pass_tuning", c_int32, [c_vp, c_int64, c_int32, c_int32, c_int32]),
    ("fs_clear_pass_tuning", c_int32, [c_vp]),
]


def exported_names():
    return [n for n, _, _ in _SIGS]


def load(path: Optional[str] = None):
    """Load libfossils.so (built in-tree by ``paper_2406_03468_amd.build``); raise if absent."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIBPATH
    if not os.path.exists(p):
        raise FileNotFoundError(f"{p} is missing: build it with `python -m paper_2406_03468_amd.build`")
    lib = ctypes.CDLL(p)
    for name, res, args in _SIGS:
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    if path is None:
        _lib = lib
    return lib


def status_string(s: int) -> str:
    try:
        return load().fs_status_string(int(s)).decode()
    except Exception:
        return f"status {s}"


def _check(s: int, allow_warn: bool = True) -> int:
    if s < 0 or (s > 0 and not allow_warn):
        detail = load().fs_last_error_detail().decode()
        raise FossilsError(s, detail)
    return s


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _colmajor(M):
    """(rows, cols) tensor with unit row stride -> leading dimension."""
    if M.dim() == 1:
        return M.shape[0]
    if M.stride(0) != 1:
        raise ValueError("matrix must be column-major (stride(0) == 1)")
    return M.stride(1) if M.shape[1] > 1 else max(M.shape[0], M.stride(1))


class Context:
    """fs_context on a torch device, bound to torch's current stream at creation."""

    def __init__(self, device: int = 0, stream=None):
        import torch

        self.lib = load()
        self.device = device
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        h = c_vp()
        _check(self.lib.fs_context_create(int(device), c_vp(stream.cuda_stream), ctypes.byref(h)))
        self.h = h

    def close(self):
        if self.h:
            self.lib.fs_context_destroy(self.h)
            self.h = None

    def __del__(self, _finalizing=sys.is_finalizing):
        # At interpreter shutdown the HIP runtime (and this module's globals) may already be gone:
        # leave the memory to the OS.
        try:
            if not _finalizing():
                self.close()
        except Exception:
            pass


def fs_options_default(m: int, n: int) -> FsOptions:
    o = FsOptions()
    _check(load().fs_options_default(int(m), int(n), ctypes.byref(o)))
    return o


def _solve(fn, ctx: Context, A, b, x, opts: Optional[FsOptions]):
    m, n = A.shape
    info = FsInfo()
    s = fn(ctx.h, int(m), int(n), c_vp(_ptr(A)), int(_colmajor(A)), c_vp(_ptr(b)), c_vp(_ptr(x)),
           ctypes.byref(opts) if opts is not None else None, ctypes.byref(info))
    return s, info


def fossils_solve(ctx: Context, A, b, x, opts: Optional[FsOptions] = None):
    s, info = _solve(load().fossils_solve, ctx, A, b, x, opts)
    _check(s)
    return s, info


def fossils_solve_noalloc(ctx: Context, A, b, x, opts: Optional[FsOptions] = None):
    """fossils_solve on the library's preallocated device array (allocates nothing)."""
    s, info = _solve(load().fossils_solve_noalloc, ctx, A, b, x, opts)
    _check(s)
    return s, info


def spir_solve(ctx: Context, A, b, x, opts: Optional[FsOptions] = None):
    s, info = _solve(load().spir_solve, ctx, A, b, x, opts)
    _check(s)
    return s, info


def spir_lsqr_solve(ctx: Context, A, b, x, opts: Optional[FsOptions] = None):
    s, info = _solve(load().spir_lsqr_solve, ctx, A, b, x, opts)
    _check(s)
    return s, info


def _complex_ld(M):
    """Leading dimension (in complex elements) of a column-major complex128 matrix or vector."""
    import torch
    if M.dtype != torch.complex128:
        raise ValueError("complex solves take complex128 tensors")
    return _colmajor(M)


def fossils_solve_complex(ctx: Context, A, b, x, opts: Optional[FsOptions] = None, method: str = "fossils"):
    """Complex least squares (complex128 column-major A (m, n), b (m,), x (n,) on the device)."""
    m, n = A.shape
    fn = {"fossils": load().fossils_solve_complex, "spir": load().spir_solve_complex}[method]
    for v in (b, x):
        _complex_ld(v)
    info = FsInfo()
    s = fn(ctx.h, int(m), int(n), c_vp(_ptr(A)), int(_complex_ld(A)), c_vp(_ptr(b)), c_vp(_ptr(x)),
           ctypes.byref(opts) if opts is not None else None, ctypes.byref(info))
    _check(s)
    return s, info


def fossils_solve_mixed(ctx: Context, A, b, x, A32=None, opts: Optional[FsOptions] = None):
    """Mixed-precision form: FP32 sketch (from A32 if given, a float32 column-major copy of A)."""
    m, n = A.shape
    info = FsInfo()
    ld32 = int(_colmajor(A32)) if A32 is not None else 0
    s = load().fossils_solve_mixed(ctx.h, int(m), int(n), c_vp(_ptr(A)), int(_colmajor(A)), c_vp(_ptr(A32)), ld32,
                                   c_vp(_ptr(b)), c_vp(_ptr(x)), ctypes.byref(opts) if opts is not None else None,
                                   ctypes.byref(info))
    _check(s)
    return s, info


def fs_to_fp32(ctx: Context, A, A32):
    m, n = A.shape
    _check(load().fs_to_fp32(ctx.h, int(m), int(n), c_vp(_ptr(A)), int(_colmajor(A)), c_vp(_ptr(A32)),
                             int(_colmajor(A32))))


def fossils_solve_multi(ctx: Context, A, B, X, opts: Optional[FsOptions] = None):
    """B: (m, k) column-major right-hand sides, X: (n, k) column-major output; returns (status, [FsInfo] * k)."""
    m, n = A.shape
    k = B.shape[1]
    if B.shape[0] != m or X.shape != (n, k):
        raise ValueError("shape mismatch")
    infos = (FsInfo * k)()
    s = load().fossils_solve_multi(ctx.h, int(m), int(n), c_vp(_ptr(A)), int(_colmajor(A)), int(k), c_vp(_ptr(B)),
                                   int(_colmajor(B)), c_vp(_ptr(X)), int(_colmajor(X)),
                                   ctypes.byref(opts) if opts is not None else None, infos)
    _check(s)
    return s, list(infos)


def fossils_solve_batched(ctx: Context, problems, opts: Optional[FsOptions] = None, check: bool = True,
                          method="fossils"):
    """problems: a list of (A, b, x) or (A, b, x, method) device tensors (A column-major (m_i, n_i), b (m_i,),
    x (n_i,) output); method "fossils" / "spir" (or an FS_METHOD_* value) for the problems that give none.
    Returns (status, [status_i], [FsInfo_i]); with check, an error status raises FossilsError."""
    k = len(problems)
    arr = (FsProblem * k)()
    codes = {"fossils": FS_METHOD_FOSSILS, "spir": FS_METHOD_SPIR}
    for i, pr in enumerate(problems):
        A, b, x = pr[:3]
        meth = pr[3] if len(pr) > 3 else method
        m, n = A.shape
        if b.shape[0] != m or x.shape[0] != n:
            raise ValueError("shape mismatch in problem %d" % i)
        arr[i] = FsProblem(int(m), int(n), c_vp(_ptr(A)), int(_colmajor(A)), c_vp(_ptr(b)), c_vp(_ptr(x)),
                           int(codes.get(meth, meth)))
    infos = (FsInfo * k)()
    sts = (c_int32 * k)()
    s = load().fossils_solve_batched(ctx.h, int(k), arr, ctypes.byref(opts) if opts is not None else None, infos,
                                     sts)
    if check:
        _check(s)
    return s, list(sts), list(infos)


class Server:
    """fs_server: worker slots draining a FIFO of solve requests (continuous batching)."""

    def __init__(self, ctx: Context, hbm_budget: int, max_slots: int = 4):
        h = c_vp()
        _check(load().fs_server_create(ctx.h, ctypes.c_size_t(int(hbm_budget)), int(max_slots), ctypes.byref(h)))
        self.h = h
        self._keep = {}  # ticket -> tensors that must outlive the solve

    def close(self):
        if self.h:
            _check(load().fs_server_destroy(self.h))
            self.h = None
            self._keep.clear()

    def __del__(self, _finalizing=sys.is_finalizing):
        try:
            if not _finalizing():
                self.close()
        except Exception:
            pass


def batched_submit(srv: Server, A, b, x, method: int = FS_METHOD_FOSSILS, opts: Optional[FsOptions] = None,
                   stream=None) -> int:
    """Enqueue a solve; it starts after the work already enqueued on `stream` (default: torch's
    current stream on A's device), which is where A and b were produced."""
    m, n = A.shape
    if stream is None:
        import torch
        stream = torch.cuda.current_stream(A.device)
    sh = stream if isinstance(stream, int) else stream.cuda_stream
    req = FsRequest(int(method), int(m), int(n), c_vp(_ptr(A)), int(_colmajor(A)), c_vp(_ptr(b)), c_vp(_ptr(x)),
                    ctypes.pointer(opts) if opts is not None else None, c_vp(sh or None))
    t = c_uint64(0)
    _check(load().batched_submit(srv.h, ctypes.byref(req), ctypes.byref(t)))
    srv._keep[t.value] = (A, b, x, opts)
    return t.value


def batched_poll(srv: Server, ticket: int):
    """(done, status, FsInfo or None)."""
    done, res, info = c_int32(0), c_int32(0), FsInfo()
    _check(load().batched_poll(srv.h, c_uint64(ticket), ctypes.byref(done), ctypes.byref(res), ctypes.byref(info)))
    if done.value:
        srv._keep.pop(ticket, None)
        return True, res.value, info
    return False, None, None


def fs_server_wait(srv: Server, ticket: int):
    _check(load().fs_server_wait(srv.h, c_uint64(ticket)))


def fs_server_ticket_times(srv: Server, ticket: int):
    a, b_, c = c_double(), c_double(), c_double()
    _check(load().fs_server_ticket_times(srv.h, c_uint64(ticket), ctypes.byref(a), ctypes.byref(b_), ctypes.byref(c)))
    return a.value, b_.value, c.value


def fs_solve_footprint(m: int, n: int, opts: Optional[FsOptions] = None) -> int:
    return int(load().fs_solve_footprint(int(m), int(n), ctypes.byref(opts) if opts is not None else None))


def fs_server_memory(srv: Server):
    """(used, peak, budget) bytes of the server's workspace ledger."""
    u, p, b_ = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_size_t()
    _check(load().fs_server_memory(srv.h, ctypes.byref(u), ctypes.byref(p), ctypes.byref(b_)))
    return u.value, p.value, b_.value


def fs_server_request_footprint(srv: Server, m: int, n: int, opts: Optional[FsOptions] = None) -> int:
    out = ctypes.c_size_t()
    _check(load().fs_server_request_footprint(srv.h, int(m), int(n), ctypes.byref(opts) if opts is not None else None,
                                              ctypes.byref(out)))
    return out.value


def fs_context_workspace(ctx: Context) -> int:
    out = ctypes.c_size_t()
    _check(load().fs_context_workspace(ctx.h, ctypes.byref(out)))
    return out.value


def fs_context_trim(ctx: Context):
    _check(load().fs_context_trim(ctx.h))


class Sketch:
    def __init__(self, ctx: Context, m: int, d: int, zeta: int, seed: int):
        self.ctx, self.m, self.d, self.zeta, self.seed = ctx, m, d, zeta, seed
        h = c_vp()
        _check(load().sketch_create(ctx.h, int(m), int(d), int(zeta), c_uint64(seed), ctypes.byref(h)))
        self.h = h

    def close(self):
        if self.h:
            load().sketch_destroy(self.h)
            self.h = None

    def __del__(self, _finalizing=sys.is_finalizing):
        try:
            if not _finalizing():
                self.close()
        except Exception:
            pass


def sketch_create(ctx: Context, m: int, d: int, zeta: int, seed: int) -> Sketch:
    return Sketch(ctx, m, d, zeta, seed)


def sketch_destroy(sk: Sketch):
    sk.close()


def sketch_indices(sk: Sketch, col0: int, ncols: int):
    import numpy as np

    rows = np.zeros(ncols * sk.zeta, dtype=np.int32)
    signs = np.zeros(ncols * sk.zeta, dtype=np.int8)
    _check(load().sketch_indices(sk.h, int(col0), int(ncols), rows.ctypes.data_as(c_vp), signs.ctypes.data_as(c_vp)))
    return rows.reshape(ncols, sk.zeta), signs.reshape(ncols, sk.zeta)


def sketch_apply(sk: Sketch, A, b, Y, colnorm2=None, scale_columns: bool = False):
    n = A.shape[1]
    _check(load().sketch_apply(sk.h, int(n), c_vp(_ptr(A)), int(_colmajor(A)), c_vp(_ptr(b)), c_vp(_ptr(Y)),
                               int(_colmajor(Y)), c_vp(_ptr(colnorm2)), int(bool(scale_columns))))


def fs_sketch_qr(ctx: Context, Y):
    d, k = Y.shape
    _check(load().fs_sketch_qr(ctx.h, int(d), int(k), c_vp(_ptr(Y)), int(_colmajor(Y))))


def fs_svd_triangular(ctx: Context, R, sigma, V) -> int:
    n = R.shape[1]
    sw = c_int32(0)
    _check(load().fs_svd_triangular(ctx.h, int(n), c_vp(_ptr(R)), int(_colmajor(R)), c_vp(_ptr(sigma)),
                                    c_vp(_ptr(V)), int(_colmajor(V)), ctypes.byref(sw)))
    return sw.value


def fs_normal_pass(ctx: Context, A, z, v):
    m, n = A.shape
    _check(load().fs_normal_pass(ctx.h, int(m), int(n), c_vp(_ptr(A)), int(_colmajor(A)), c_vp(_ptr(z)),
                                 c_vp(_ptr(v))))


def fs_residual_pass(ctx: Context, A, b, x, g) -> float:
    m, n = A.shape
    r2 = c_double(0.0)
    _check(load().fs_residual_pass(ctx.h, int(m), int(n), c_vp(_ptr(A)), int(_colmajor(A)), c_vp(_ptr(b)),
                                   c_vp(_ptr(x)), c_vp(_ptr(g)), ctypes.byref(r2)))
    return r2.value


def fs_trsv(ctx: Context, R, y, x, transpose: bool = False):
    n = R.shape[1]
    _check(load().fs_trsv(ctx.h, int(n), c_vp(_ptr(R)), int(_colmajor(R)), int(bool(transpose)), c_vp(_ptr(y)),
                          c_vp(_ptr(x))))


def fs_triangular_inverse(ctx: Context, R, X):
    """X = R^{-1} (upper-triangular R); X: n x n, column-major with leading dimension n."""
    n = R.shape[1]
    if tuple(X.shape) != (n, n) or _colmajor(X) != n:
        raise ValueError("X must be n x n, column-major with leading dimension n")
    _check(load().fs_triangular_inverse(ctx.h, int(n), c_vp(_ptr(R)), int(_colmajor(R)), c_vp(_ptr(X))))


def fs_time_normal_pass(ctx: Context, A, z, v, repeats: int = 20):
    """(ms per pass incl. reduction, ms of the fused kernel alone), averaged over `repeats`."""
    m, n = A.shape
    t, tk = c_double(0.0), c_double(0.0)
    _check(load().fs_time_normal_pass(ctx.h, int(m), int(n), c_vp(_ptr(A)), int(_colmajor(A)), c_vp(_ptr(z)),
                                      c_vp(_ptr(v)), int(repeats), ctypes.byref(t), ctypes.byref(tk)))
    return t.value, tk.value


def fs_tune_pass(ctx: Context, A, z, v, repeats: int = 5):
    """Time every admissible (tile height, work-group count) of the fused pass on A and keep the
    fastest in the context for this (n, m-bucket); returns (H, G, ms per pass)."""
    m, n = A.shape
    H, G, ms = c_int32(0), c_int32(0), c_double(0.0)
    _check(load().fs_tune_pass(ctx.h, int(m), int(n), c_vp(_ptr(A)), int(_colmajor(A)), c_vp(_ptr(z)), c_vp(_ptr(v)),
                               int(repeats), ctypes.byref(H), ctypes.byref(G), ctypes.byref(ms)))
    return H.value, G.value, ms.value


def fs_set_pass_tuning(ctx: Context, m: int, n: int, H: int, G: int):
    _check(load().fs_set_pass_tuning(ctx.h, int(m), int(n), int(H), int(G)))


def fs_clear_pass_tuning(ctx: Context):
    _check(load().fs_clear_pass_tuning(ctx.h))
