"""Shared helpers for the tests: error norm, host/device copies, and an
independent numpy evaluation of the low-order velocity (numpy's FFT of the
definition) for meshes where the oracle's direct DFT sums would take hours."""
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


def fft_reference(n1, n2, z, w, L1=2.0, L2=2.0):
    """u = 1/2 (R1 w1 + R2 w2) n^ by numpy's FFT (the definition's symbols,
    Nyquist modes zeroed along their own axis); n^ from the oracle's
    tangents."""
    import oracle
    W1 = np.fft.fft2(w[0].reshape(n2, n1))
    W2 = np.fft.fft2(w[1].reshape(n2, n1))
    K1 = 2 * np.pi * np.fft.fftfreq(n1, 1.0 / n1)[None, :] / L1 + 0 * np.arange(n2)[:, None]
    K2 = 2 * np.pi * np.fft.fftfreq(n2, 1.0 / n2)[:, None] / L2 + 0 * np.arange(n1)[None, :]
    KK = np.hypot(K1, K2)
    with np.errstate(invalid="ignore", divide="ignore"):
        c1 = np.where(KK > 0, K1 / KK, 0.0)
        c2 = np.where(KK > 0, K2 / KK, 0.0)
    c1[:, n1 // 2] = 0.0
    c2[n2 // 2, :] = 0.0
    S = np.real(np.fft.ifft2(0.5j * (c1 * W1 + c2 * W2))).ravel()
    t1, t2 = oracle.tangents(oracle.Problem(n1, n2, eps=1.0 / n1, period1=L1, period2=L2), z)
    nrm = np.cross(t1.T, t2.T).T
    return S * (nrm / np.linalg.norm(nrm, axis=0))
