"""Helpers shared by the GPU parity tests (torch for device memory only)."""
from __future__ import annotations

import math

import numpy as np


def torch_dev():
    import torch
    if not torch.cuda.is_available():
        import pytest
        pytest.skip("no GPU")
    return torch


def to_dev(a: np.ndarray, dtype=None):
    torch = torch_dev()
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def to_host(t) -> np.ndarray:
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def bf16_round(a: np.ndarray) -> np.ndarray:
    """Round float64 values to bfloat16 (ties to even) via float32 bit patterns (exact for values already
    representable in float32)."""
    f = a.astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def log_natural(f_eps: np.ndarray, eps: float) -> np.ndarray:
    """f = eps * log a  ->  log a."""
    return f_eps / eps
