"""Helpers shared by the GPU parity tests."""
import sys

import numpy as np


def announce(msg: str) -> None:
    """Name the case before any GPU work, so a failed run says which one."""
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def dev_f(a: np.ndarray, dtype=None):
    """Column-major device tensor from a numpy array."""
    import torch
    from paper_1803_01982_amd import fortran
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return fortran(t.cuda())


def host(t) -> np.ndarray:
    return t.detach().cpu().numpy()


def rel(a, b) -> float:
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))
