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
