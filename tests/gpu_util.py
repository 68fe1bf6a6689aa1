"""Helpers for the GPU tests: column-major device tensors and a shared context."""

import numpy as np


def dev_colmajor(M, ld=None):
    """numpy (rows, cols) -> torch float64 cuda tensor, column-major, leading dimension ld."""
    import torch

    M = np.asarray(M, dtype=np.float64)
    rows, cols = M.shape
    ld = ld or rows
    buf = torch.zeros((cols, ld), dtype=torch.float64, device="cuda")
    buf[:, :rows] = torch.as_tensor(np.ascontiguousarray(M.T), device="cuda")
    return buf.t()[:rows, :]  # (rows, cols) view with strides (1, ld)


def dev_vec(v):
    import torch

    return torch.as_tensor(np.asarray(v, dtype=np.float64)).to("cuda")


def host(t):
    return t.detach().cpu().numpy()


def empty_colmajor(rows, cols, ld=None):
    import torch

    ld = ld or rows
    return torch.zeros((cols, ld), dtype=torch.float64, device="cuda").t()[:rows, :]


def assert_stats(info, condest, normest=None, rel=1e-9):
    """normest / condest of a GPU solve against reference values.  Exact (to `rel`) when the SVD of R
    finished; when the solve stopped before needing it (FS_FLAG_SVD_ABANDONED) they are lower bounds
    from diag(R) and a few power / inverse iteration steps: at most the true value, within 4x."""
    abandoned = bool(info.flags & 16)
    for got, ref in ((info.condest, condest), (info.normest, normest)):
        if ref is None:
            continue
        if abandoned:
            assert ref / 4 <= got <= ref * (1 + 1e-6), (got, ref, "lower bound")
        else:
            assert abs(got - ref) <= rel * ref, (got, ref)
