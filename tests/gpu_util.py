"""Shared helpers for the GPU parity tests."""
import numpy as np
import pytest
import torch

TAU, G = 0.05, 5.0


def require_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


def to_dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a)).cuda()
    return t.to(dtype) if dtype is not None else t


def to_host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rel_err(a, b):
    """max |a - b| / max |b| (element-wise comparison, scaled by the output size)."""
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def say(*args):
    print(*args, flush=True)
