"""Plain FP64 CPU oracle for the Z-Model high-order step (test infrastructure).

Only the test suite, the package smoke check and the benchmark's CPU-baseline
leg may import this package.  It shares no code with the GPU library.

All arrays are float64 numpy arrays in structure-of-arrays plane layout:
``z`` has shape (3, n2, n1) (or (3, N)), ``w`` has shape (2, n2, n1); point
index p = i2 * n1 + i1.  See ``zm_oracle.c`` for the definitions.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libzm_oracle.so")
# The mutation tests point this at a deliberately broken build of the oracle.
_LIB_PATH = os.environ.get("ZMO_ORACLE_LIB", _LIB_PATH)


class _Problem(ctypes.Structure):
    _fields_ = [
        ("n1", ctypes.c_int32), ("n2", ctypes.c_int32),
        ("images", ctypes.c_int32), ("model", ctypes.c_int32),
        ("period1", ctypes.c_double), ("period2", ctypes.c_double),
        ("atwood", ctypes.c_double), ("gravity", ctypes.c_double),
        ("eps", ctypes.c_double), ("nu", ctypes.c_double), ("dt", ctypes.c_double),
        ("cutoff", ctypes.c_double),
        ("boundary", ctypes.c_int32), ("pad_", ctypes.c_int32),
    ]


@dataclass
class Problem:
    """Mesh and model parameters (same meaning as the GPU library's)."""
    n1: int
    n2: int
    eps: float
    atwood: float = 0.5
    gravity: float = 1.0
    dt: float = 1e-3
    nu: float = 0.0
    images: int = 0
    period1: float = 2.0
    period2: float = 2.0
    cutoff: float = 0.0       # > 0: cutoff BR solver (3D distance)
    model: int = 0            # 0: high order (BR sum), 1: low order (FFT velocity),
                              # 2: medium order (BR moves the sheet, FFT velocity in V)
    boundary: int = 0         # 0: periodic, 1: free (extrapolated ghosts, no images)

    def c(self) -> _Problem:
        return _Problem(self.n1, self.n2, self.images, self.model, self.period1, self.period2,
                        self.atwood, self.gravity, self.eps, self.nu, self.dt, self.cutoff,
                        self.boundary, 0)

    @property
    def n(self) -> int:
        return self.n1 * self.n2


_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(_LIB_PATH)
    P = ctypes.POINTER(_Problem)
    D = ctypes.POINTER(ctypes.c_double)
    I64 = ctypes.POINTER(ctypes.c_int64)
    lib.zmo_tangents.argtypes = [P, D, D, D]
    lib.zmo_tangents.restype = None
    lib.zmo_surface.argtypes = [P, D, D, D, D, D, D]
    lib.zmo_surface.restype = None
    lib.zmo_laplacian.argtypes = [P, D, D]
    lib.zmo_laplacian.restype = None
    lib.zmo_br_velocity.argtypes = [P, D, D, ctypes.c_int64, I64, D, ctypes.c_int]
    lib.zmo_br_velocity.restype = ctypes.c_int
    lib.zmo_br_from_gamma.argtypes = [P, D, D, ctypes.c_int64, I64, D, ctypes.c_int]
    lib.zmo_br_from_gamma.restype = ctypes.c_int
    lib.zmo_rhs.argtypes = [P, D, D, D, D, ctypes.c_int]
    lib.zmo_rhs.restype = ctypes.c_int
    lib.zmo_rhs_sampled.argtypes = [P, D, D, ctypes.c_int64, I64, D, D, ctypes.c_int]
    lib.zmo_rhs_sampled.restype = ctypes.c_int
    lib.zmo_wt_sampled.argtypes = [P, D, D, D, ctypes.c_int64, I64, D]
    lib.zmo_wt_sampled.restype = ctypes.c_int
    lib.zmo_rk3_step.argtypes = [P, D, D, ctypes.c_int, ctypes.c_int]
    lib.zmo_rk3_step.restype = ctypes.c_int
    _lib = lib
    return lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _planes(a, ncomp: int, n: int) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64)).reshape(ncomp, n)
    return a


def _targets(targets):
    if targets is None:
        return 0, None, None
    t = np.ascontiguousarray(np.asarray(targets, dtype=np.int64).ravel())
    return t.size, t, t.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))


def tangents(P: Problem, z):
    lib = _load()
    z = _planes(z, 3, P.n)
    t1 = np.empty((3, P.n)); t2 = np.empty((3, P.n))
    lib.zmo_tangents(ctypes.byref(P.c()), _dp(z), _dp(t1), _dp(t2))
    return t1, t2


def surface(P: Problem, z, w):
    """Returns (T1, T2, gamma, q): tangents, BR source strength, squared
    tangential-velocity jump."""
    lib = _load()
    z = _planes(z, 3, P.n); w = _planes(w, 2, P.n)
    t1 = np.empty((3, P.n)); t2 = np.empty((3, P.n)); g = np.empty((3, P.n)); q = np.empty(P.n)
    lib.zmo_surface(ctypes.byref(P.c()), _dp(z), _dp(w), _dp(t1), _dp(t2), _dp(g), _dp(q))
    return t1, t2, g, q


def laplacian(P: Problem, f):
    lib = _load()
    f = np.ascontiguousarray(np.asarray(f, dtype=np.float64).ravel())
    out = np.empty(P.n)
    lib.zmo_laplacian(ctypes.byref(P.c()), _dp(f), _dp(out))
    return out


def br_velocity(P: Problem, z, w, targets=None, threads: int = 0) -> np.ndarray:
    """BR velocity, shape (3, ntargets) (all points when targets is None)."""
    lib = _load()
    z = _planes(z, 3, P.n); w = _planes(w, 2, P.n)
    nt, t, tp = _targets(targets)
    u = np.empty((3, nt if t is not None else P.n))
    rc = lib.zmo_br_velocity(ctypes.byref(P.c()), _dp(z), _dp(w), nt, tp, _dp(u), threads)
    if rc:
        raise ValueError("oracle: bad arguments to br_velocity")
    return u


def br_from_gamma(P: Problem, z, gamma, targets=None, threads: int = 0) -> np.ndarray:
    lib = _load()
    z = _planes(z, 3, P.n); g = _planes(gamma, 3, P.n)
    nt, t, tp = _targets(targets)
    u = np.empty((3, nt if t is not None else P.n))
    rc = lib.zmo_br_from_gamma(ctypes.byref(P.c()), _dp(z), _dp(g), nt, tp, _dp(u), threads)
    if rc:
        raise ValueError("oracle: bad arguments to br_from_gamma")
    return u


def rhs(P: Problem, z, w, threads: int = 0):
    """F(z, w) = (z_t, w_t), shapes (3, N) and (2, N)."""
    lib = _load()
    z = _planes(z, 3, P.n); w = _planes(w, 2, P.n)
    zt = np.empty((3, P.n)); wt = np.empty((2, P.n))
    rc = lib.zmo_rhs(ctypes.byref(P.c()), _dp(z), _dp(w), _dp(zt), _dp(wt), threads)
    if rc:
        raise ValueError("oracle: bad arguments to rhs")
    return zt, wt


def rhs_sampled(P: Problem, z, w, targets, threads: int = 0):
    """F at the listed point indices: shapes (3, nt) and (2, nt)."""
    lib = _load()
    z = _planes(z, 3, P.n); w = _planes(w, 2, P.n)
    nt, t, tp = _targets(targets)
    zt = np.empty((3, nt)); wt = np.empty((2, nt))
    rc = lib.zmo_rhs_sampled(ctypes.byref(P.c()), _dp(z), _dp(w), nt, tp, _dp(zt), _dp(wt), threads)
    if rc:
        raise ValueError("oracle: bad arguments to rhs_sampled")
    return zt, wt


def wt_sampled(P: Problem, z, w, u, targets):
    """The vorticity derivative at the listed point indices, shape (2, nt),
    with the velocity in V given as the full field ``u`` (shape (3, N)): the
    medium-order w_t when ``u`` is the FFT velocity."""
    lib = _load()
    z = _planes(z, 3, P.n); w = _planes(w, 2, P.n); u = _planes(u, 3, P.n)
    nt, t, tp = _targets(targets)
    wt = np.empty((2, nt))
    rc = lib.zmo_wt_sampled(ctypes.byref(P.c()), _dp(z), _dp(w), _dp(u), nt, tp, _dp(wt))
    if rc:
        raise ValueError("oracle: bad arguments to wt_sampled")
    return wt


def rk3(P: Problem, z, w, nsteps: int, threads: int = 0):
    """Advance copies of (z, w) by nsteps SSP-RK3 steps; returns (z, w)."""
    lib = _load()
    z = _planes(z, 3, P.n).copy(); w = _planes(w, 2, P.n).copy()
    rc = lib.zmo_rk3_step(ctypes.byref(P.c()), _dp(z), _dp(w), int(nsteps), threads)
    if rc:
        raise ValueError("oracle: bad arguments to rk3")
    return z, w
