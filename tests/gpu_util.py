"""Helpers shared by the GPU parity tests (no method arithmetic here)."""
import numpy as np


def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU test needs a HIP device"
    return torch


def to_dev(a, dtype=None):
    torch = torch_cuda()
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def banner(msg):
    print("[gpu] " + msg, flush=True)
