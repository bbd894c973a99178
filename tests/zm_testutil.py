"""Shared helpers for the tests (no method arithmetic)."""
import numpy as np


def relerr(a, b):
    """Normwise relative error: max |a - b| / max |b|."""
    a = np.asarray(a); b = np.asarray(b)
    den = np.max(np.abs(b))
    return float(np.max(np.abs(a - b)) / den) if den > 0 else float(np.max(np.abs(a)))


def to_dev(a, device):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64).ravel()).to(device)


def to_host(t, shape=None):
    a = t.detach().cpu().numpy()
    return a.reshape(shape) if shape is not None else a
