"""Helpers for the GPU tests: device placement of the seeded inputs and
readable per-case logging (the case is printed and flushed before each launch)."""
from __future__ import annotations

import sys

import numpy as np


def log(msg: str):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def torch_dev():
    import torch
    if not torch.cuda.is_available():
        import pytest
        pytest.skip("no HIP device")
    return torch


def to_dev(a: np.ndarray, dtype=None):
    torch = torch_dev()
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to("cuda:0")


def to_host(t) -> np.ndarray:
    return t.detach().to("cpu").numpy()


def rel_err(a, b) -> float:
    a = np.asarray(a, dtype=np.complex128)
    b = np.asarray(b, dtype=np.complex128)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def max_rel_elem(a, b) -> float:
    """max |a - b| / max |b| (element-wise error against the field's scale)."""
    a = np.asarray(a, dtype=np.complex128)
    b = np.asarray(b, dtype=np.complex128)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))
