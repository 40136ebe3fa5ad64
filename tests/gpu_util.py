"""Helpers for the GPU tests: device buffers through torch (memory only) and the library."""
import numpy as np
import pytest


def require_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    return torch


def dev(a, dtype=None):
    """Copy a numpy array to the GPU (torch tensor) and wait for the copy."""
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a if dtype is None else a.astype(dtype))).cuda()
    torch.cuda.synchronize()
    return t


def empty(n, dtype):
    import torch
    t = torch.zeros(n, dtype=dtype, device="cuda")
    torch.cuda.synchronize()
    return t


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()
