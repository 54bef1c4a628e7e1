"""Helpers for the GPU parity tests (no spreading/interpolation arithmetic here)."""
import sys

import numpy as np
import torch


def say(msg):
    """Name the case before a GPU step, flushed, so a failing run shows where it was."""
    sys.stdout.write(f"[gpu] {msg}\n")
    sys.stdout.flush()


def to_dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def to_host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def normwise(a, b):
    """||a - b||_inf / ||b||_inf (0 when both vanish)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.abs(b).max() if b.size else 0.0
    num = np.abs(a - b).max() if b.size else 0.0
    if den == 0.0:
        return float(num)
    return float(num / den)


TOL = {torch.float64: 1e-12, torch.float32: 2e-6}
