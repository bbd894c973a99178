"""ctypes binding of libzm.so (include/zm.h): argument marshalling only.

Every step of the computation runs in the HIP library; this module only
converts torch tensors to device pointers and status codes to exceptions.
Names follow the C entry points (``zm_create`` -> ``create`` etc.).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

HERE = os.path.dirname(os.path.abspath(__file__))
# ZM_LIBRARY selects another build of the same library (the host-sanitizer
# test loads one); by default the in-tree build is used.
LIB_PATH = os.environ.get("ZM_LIBRARY", os.path.join(HERE, "libzm.so"))

ZM_OK = 0
ZM_ERR_INVALID_ARG = -1
ZM_ERR_UNSUPPORTED = -2
ZM_ERR_WORKSPACE = -3
ZM_ERR_HIP = -4
ZM_ERR_NONFINITE = -5
ZM_ERR_CAPACITY = -6

ZM_FP64 = 0
ZM_FP32_PAIRS = 1
ZM_MODEL_HIGH = 0
ZM_MODEL_LOW = 1
ZM_MODEL_MEDIUM = 2
ZM_BOUNDARY_PERIODIC = 0
ZM_BOUNDARY_FREE = 1
ZM_FLAG_CHECK_FINITE = 0x1
ZM_FLAG_GRAPH = 0x2
ZM_CUT_PATH_CELLS = 1
ZM_CUT_PATH_WINDOW = 2
ZM_CUT_PATH_STENCIL = 4
NOALLOC_SCRATCH_BYTES = 64 * 1024 * 1024   # ZM_NOALLOC_SCRATCH_BYTES

KERNELS = ("surface", "pairs", "ties", "reduce", "update", "cells", "fft")


class ZMError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"zm status {status}: {message}")
        self.status = status


class zm_params(ctypes.Structure):
    _fields_ = [
        ("n1", ctypes.c_int32), ("n2", ctypes.c_int32),
        ("period1", ctypes.c_double), ("period2", ctypes.c_double),
        ("atwood", ctypes.c_double), ("gravity", ctypes.c_double),
        ("eps", ctypes.c_double), ("nu", ctypes.c_double), ("dt", ctypes.c_double),
        ("precision", ctypes.c_int32), ("image_layers", ctypes.c_int32),
        ("flags", ctypes.c_uint32), ("model", ctypes.c_int32),
        ("cutoff", ctypes.c_double),
        ("boundary", ctypes.c_int32), ("reserved", ctypes.c_int32),
    ]


class zm_cutoff_info(ctypes.Structure):
    _fields_ = [("cells1", ctypes.c_int32), ("cells2", ctypes.c_int32),
                ("cells_per_cutoff", ctypes.c_int32), ("block_cells", ctypes.c_int32),
                ("slots", ctypes.c_int32), ("paths", ctypes.c_int32),
                ("pairs_tested", ctypes.c_int64), ("pairs_accepted", ctypes.c_int64)]


class zm_launch_info(ctypes.Structure):
    _fields_ = [
        ("targets_per_lane", ctypes.c_int32), ("patch_cols", ctypes.c_int32),
        ("patch_rows", ctypes.c_int32), ("source_splits", ctypes.c_int32),
        ("workgroups", ctypes.c_int32), ("threads_per_group", ctypes.c_int32),
        ("pairs_per_eval", ctypes.c_int64),
    ]


class zm_kernel_stats(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int64), ("total_ms", ctypes.c_double)]


ZM_REQ_UNKNOWN = -1
ZM_REQ_QUEUED = 0
ZM_REQ_LIVE = 1
ZM_REQ_FINISHED = 2
ZM_REQ_FAILED = 3


class zm_step_record(ctypes.Structure):
    _fields_ = [("id", ctypes.c_int64), ("steps_done", ctypes.c_int32), ("state", ctypes.c_int32),
                ("iteration_ms", ctypes.c_double)]


class zm_pool_stats(ctypes.Structure):
    _fields_ = [("queued", ctypes.c_int32), ("live", ctypes.c_int32), ("finished", ctypes.c_int32),
                ("iterations", ctypes.c_int32), ("used_bytes", ctypes.c_int64),
                ("budget_bytes", ctypes.c_int64), ("pairs_done", ctypes.c_int64)]


class zm_pair_tuning(ctypes.Structure):
    _fields_ = [("targets_per_lane", ctypes.c_int32), ("source_splits", ctypes.c_int32)]


class zm_batch_info(ctypes.Structure):
    _fields_ = [("count", ctypes.c_int32), ("work_items", ctypes.c_int32 * 2),
                ("persistent_groups", ctypes.c_int32), ("pairs_per_step", ctypes.c_int64)]


# names declared in include/zm.h, in order
EXPORTS = (
    "zm_workspace_bytes", "zm_create", "zm_init_state", "zm_br_velocity", "zm_rhs",
    "zm_step", "zm_get_state", "zm_destroy", "zm_status_string", "zm_last_error",
    "zm_get_launch_info", "zm_profile_enable", "zm_profile_read", "zm_cutoff_info_get",
    "zm_tuning_set", "zm_tuning_get", "zm_autotune_workspace_bytes", "zm_autotune",
    "zm_batch_autotune_workspace_bytes", "zm_batch_autotune",
    "zm_batch_workspace_bytes", "zm_batch_create", "zm_batch_init_state", "zm_batch_get_state",
    "zm_batch_step", "zm_batch_get_info", "zm_batch_destroy", "zm_batch_last_error",
    "zm_pool_workspace_bytes", "zm_pool_request_bytes", "zm_pool_create", "zm_pool_submit",
    "zm_pool_iterate", "zm_pool_query", "zm_pool_fetch", "zm_pool_release", "zm_pool_cancel",
    "zm_pool_get_stats", "zm_pool_destroy", "zm_pool_last_error",
    "zm_br_velocity_noalloc", "zm_abi_version",
)

_lib = None


def load(path: str = LIB_PATH):
    """Load libzm.so; raises ImportError if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with "
                          "`python paper_2406_05490_amd/build.py` (no fallback exists)")
    # PyTorch ships its own HIP runtime.  Loading torch first makes the
    # library's libamdhip64.so.7 dependency resolve to that same runtime, so
    # torch's streams and allocations are valid in the library (a second
    # HIP/HSA runtime in the process would not see torch's objects).
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    P = ctypes.POINTER(zm_params)
    vp = ctypes.c_void_p
    lib.zm_workspace_bytes.argtypes = [P]
    lib.zm_workspace_bytes.restype = ctypes.c_size_t
    lib.zm_create.argtypes = [ctypes.POINTER(vp), P, vp, ctypes.c_size_t, vp]
    lib.zm_create.restype = ctypes.c_int32
    lib.zm_init_state.argtypes = [vp, vp, vp]
    lib.zm_init_state.restype = ctypes.c_int32
    lib.zm_br_velocity.argtypes = [vp, vp, vp, vp]
    lib.zm_br_velocity.restype = ctypes.c_int32
    lib.zm_rhs.argtypes = [vp, vp, vp, vp, vp]
    lib.zm_rhs.restype = ctypes.c_int32
    lib.zm_step.argtypes = [vp, ctypes.c_int32]
    lib.zm_step.restype = ctypes.c_int32
    lib.zm_get_state.argtypes = [vp, vp, vp]
    lib.zm_get_state.restype = ctypes.c_int32
    lib.zm_destroy.argtypes = [vp]
    lib.zm_destroy.restype = ctypes.c_int32
    lib.zm_status_string.argtypes = [ctypes.c_int32]
    lib.zm_status_string.restype = ctypes.c_char_p
    lib.zm_last_error.argtypes = [vp]
    lib.zm_last_error.restype = ctypes.c_char_p
    lib.zm_get_launch_info.argtypes = [vp, ctypes.POINTER(zm_launch_info)]
    lib.zm_get_launch_info.restype = ctypes.c_int32
    lib.zm_profile_enable.argtypes = [vp, ctypes.c_int32]
    lib.zm_profile_enable.restype = ctypes.c_int32
    lib.zm_profile_read.argtypes = [vp, ctypes.POINTER(zm_kernel_stats)]
    lib.zm_profile_read.restype = ctypes.c_int32
    lib.zm_cutoff_info_get.argtypes = [vp, ctypes.POINTER(zm_cutoff_info)]
    lib.zm_cutoff_info_get.restype = ctypes.c_int32
    T = ctypes.POINTER(zm_pair_tuning)
    lib.zm_tuning_set.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, T]
    lib.zm_tuning_set.restype = ctypes.c_int32
    lib.zm_tuning_get.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, T]
    lib.zm_tuning_get.restype = ctypes.c_int32
    lib.zm_autotune_workspace_bytes.argtypes = [P]
    lib.zm_autotune_workspace_bytes.restype = ctypes.c_size_t
    lib.zm_autotune.argtypes = [P, vp, ctypes.c_size_t, vp, T, ctypes.POINTER(ctypes.c_double)]
    lib.zm_autotune.restype = ctypes.c_int32
    lib.zm_batch_autotune_workspace_bytes.argtypes = [P, ctypes.c_int32]
    lib.zm_batch_autotune_workspace_bytes.restype = ctypes.c_size_t
    lib.zm_batch_autotune.argtypes = [P, ctypes.c_int32, vp, ctypes.c_size_t, vp, T,
                                      ctypes.POINTER(ctypes.c_double)]
    lib.zm_batch_autotune.restype = ctypes.c_int32
    lib.zm_batch_workspace_bytes.argtypes = [P, ctypes.c_int32]
    lib.zm_batch_workspace_bytes.restype = ctypes.c_size_t
    lib.zm_batch_create.argtypes = [ctypes.POINTER(vp), P, ctypes.c_int32, ctypes.c_uint32, vp,
                                    ctypes.c_size_t, vp]
    lib.zm_batch_create.restype = ctypes.c_int32
    lib.zm_batch_init_state.argtypes = [vp, ctypes.c_int32, vp, vp]
    lib.zm_batch_init_state.restype = ctypes.c_int32
    lib.zm_batch_get_state.argtypes = [vp, ctypes.c_int32, vp, vp]
    lib.zm_batch_get_state.restype = ctypes.c_int32
    lib.zm_batch_step.argtypes = [vp, ctypes.c_int32]
    lib.zm_batch_step.restype = ctypes.c_int32
    lib.zm_batch_get_info.argtypes = [vp, ctypes.POINTER(zm_batch_info)]
    lib.zm_batch_get_info.restype = ctypes.c_int32
    lib.zm_batch_destroy.argtypes = [vp]
    lib.zm_batch_destroy.restype = ctypes.c_int32
    lib.zm_batch_last_error.argtypes = [vp]
    lib.zm_batch_last_error.restype = ctypes.c_char_p
    I64P = ctypes.POINTER(ctypes.c_int64)
    I32P = ctypes.POINTER(ctypes.c_int32)
    lib.zm_pool_workspace_bytes.argtypes = [ctypes.c_size_t]
    lib.zm_pool_workspace_bytes.restype = ctypes.c_size_t
    lib.zm_pool_request_bytes.argtypes = [P]
    lib.zm_pool_request_bytes.restype = ctypes.c_size_t
    lib.zm_pool_create.argtypes = [ctypes.POINTER(vp), ctypes.c_size_t, ctypes.c_uint32, vp,
                                   ctypes.c_size_t, vp]
    lib.zm_pool_create.restype = ctypes.c_int32
    lib.zm_pool_submit.argtypes = [vp, P, vp, vp, ctypes.c_int32, I64P]
    lib.zm_pool_submit.restype = ctypes.c_int32
    lib.zm_pool_iterate.argtypes = [vp, ctypes.POINTER(zm_step_record), ctypes.c_int32, I32P]
    lib.zm_pool_iterate.restype = ctypes.c_int32
    lib.zm_pool_query.argtypes = [vp, ctypes.c_int64, I32P, I32P]
    lib.zm_pool_query.restype = ctypes.c_int32
    lib.zm_pool_fetch.argtypes = [vp, ctypes.c_int64, vp, vp]
    lib.zm_pool_fetch.restype = ctypes.c_int32
    lib.zm_pool_release.argtypes = [vp, ctypes.c_int64]
    lib.zm_pool_release.restype = ctypes.c_int32
    lib.zm_pool_cancel.argtypes = [vp, ctypes.c_int64]
    lib.zm_pool_cancel.restype = ctypes.c_int32
    lib.zm_pool_get_stats.argtypes = [vp, ctypes.POINTER(zm_pool_stats)]
    lib.zm_pool_get_stats.restype = ctypes.c_int32
    lib.zm_pool_destroy.argtypes = [vp]
    lib.zm_pool_destroy.restype = ctypes.c_int32
    lib.zm_pool_last_error.argtypes = [vp]
    lib.zm_pool_last_error.restype = ctypes.c_char_p
    lib.zm_br_velocity_noalloc.argtypes = [P, vp, vp, vp, vp]
    lib.zm_br_velocity_noalloc.restype = ctypes.c_int32
    lib.zm_abi_version.argtypes = []
    lib.zm_abi_version.restype = ctypes.c_int32
    _lib = lib
    return lib


@dataclass
class Params:
    """Python mirror of zm_params."""
    n1: int
    n2: int
    eps: float
    atwood: float = 0.5
    gravity: float = 1.0
    dt: float = 1e-3
    nu: float = 0.0
    period1: float = 2.0
    period2: float = 2.0
    precision: int = ZM_FP64
    image_layers: int = 0
    flags: int = 0
    cutoff: float = 0.0       # > 0: cutoff BR solver with this 3D distance
    model: int = ZM_MODEL_HIGH
    boundary: int = ZM_BOUNDARY_PERIODIC

    def c(self) -> zm_params:
        return zm_params(self.n1, self.n2, self.period1, self.period2, self.atwood,
                         self.gravity, self.eps, self.nu, self.dt, self.precision,
                         self.image_layers, self.flags, self.model, self.cutoff,
                         self.boundary, 0)

    @property
    def n(self) -> int:
        return self.n1 * self.n2


def status_string(status: int) -> str:
    return load().zm_status_string(status).decode()


def workspace_bytes(p: Params) -> int:
    return int(load().zm_workspace_bytes(ctypes.byref(p.c())))


def _ptr(t) -> int:
    return 0 if t is None else int(t.data_ptr())


def _check_f64_planes(t, planes: int, n: int, name: str):
    import torch
    if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous() or t.numel() != planes * n:
        raise ValueError(f"{name}: need a contiguous float64 CUDA tensor of {planes} x {n} values")


class Context:
    """One zm_ctx with a workspace tensor it keeps alive."""

    def __init__(self, p: Params, stream=None, device=None):
        import torch
        self.lib = load()
        self.params = p
        dev = torch.device("cuda", torch.cuda.current_device()) if device is None else device
        nbytes = workspace_bytes(p)
        if nbytes == 0:
            # let the library say why (invalid or unsupported parameters)
            h = ctypes.c_void_p()
            st = self.lib.zm_create(ctypes.byref(h), ctypes.byref(p.c()), None, 0, None)
            raise ZMError(st if st != ZM_OK else ZM_ERR_INVALID_ARG,
                          self.lib.zm_last_error(None).decode() or "invalid parameters")
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        self.stream = torch.cuda.current_stream(dev) if stream is None else stream
        h = ctypes.c_void_p()
        with torch.cuda.device(dev):
            st = self.lib.zm_create(ctypes.byref(h), ctypes.byref(p.c()),
                                    self.workspace.data_ptr(), nbytes, self.stream.cuda_stream)
        if st != ZM_OK:
            raise ZMError(st, self.lib.zm_last_error(None).decode())
        self.handle = h

    def _raise(self, st):
        if st != ZM_OK:
            raise ZMError(st, self.lib.zm_last_error(self.handle).decode())

    def init_state(self, z, w):
        _check_f64_planes(z, 3, self.params.n, "z"); _check_f64_planes(w, 2, self.params.n, "w")
        self._raise(self.lib.zm_init_state(self.handle, _ptr(z), _ptr(w)))

    def get_state(self, z, w):
        _check_f64_planes(z, 3, self.params.n, "z"); _check_f64_planes(w, 2, self.params.n, "w")
        self._raise(self.lib.zm_get_state(self.handle, _ptr(z), _ptr(w)))

    def br_velocity(self, z, w, u):
        _check_f64_planes(z, 3, self.params.n, "z"); _check_f64_planes(w, 2, self.params.n, "w")
        _check_f64_planes(u, 3, self.params.n, "u")
        self._raise(self.lib.zm_br_velocity(self.handle, _ptr(z), _ptr(w), _ptr(u)))

    def rhs(self, z, w, zt, wt):
        for t, k, nm in ((z, 3, "z"), (w, 2, "w"), (zt, 3, "zt"), (wt, 2, "wt")):
            _check_f64_planes(t, k, self.params.n, nm)
        self._raise(self.lib.zm_rhs(self.handle, _ptr(z), _ptr(w), _ptr(zt), _ptr(wt)))

    def step(self, nsteps: int):
        self._raise(self.lib.zm_step(self.handle, int(nsteps)))

    def launch_info(self) -> zm_launch_info:
        info = zm_launch_info()
        self._raise(self.lib.zm_get_launch_info(self.handle, ctypes.byref(info)))
        return info

    def profile_enable(self, on: bool = True):
        self._raise(self.lib.zm_profile_enable(self.handle, 1 if on else 0))

    def profile_read(self) -> dict:
        arr = (zm_kernel_stats * len(KERNELS))()
        self._raise(self.lib.zm_profile_read(self.handle, arr))
        return {k: (int(arr[i].launches), float(arr[i].total_ms)) for i, k in enumerate(KERNELS)}

    def cutoff_info(self) -> zm_cutoff_info:
        info = zm_cutoff_info()
        self._raise(self.lib.zm_cutoff_info_get(self.handle, ctypes.byref(info)))
        return info

    def destroy(self):
        if getattr(self, "handle", None) is not None:
            st = self.lib.zm_destroy(self.handle)
            self.handle = None
            if st != ZM_OK:
                raise ZMError(st, "destroy")

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def tuning_set(n1: int, n2: int, precision: int, targets_per_lane=None, source_splits=None):
    """Set the launch shape for a mesh size (None, None: remove the entry)."""
    lib = load()
    if targets_per_lane is None:
        st = lib.zm_tuning_set(n1, n2, precision, None)
    else:
        t = zm_pair_tuning(int(targets_per_lane), int(source_splits))
        st = lib.zm_tuning_set(n1, n2, precision, ctypes.byref(t))
    if st != ZM_OK:
        raise ZMError(st, "tuning_set")


def tuning_get(n1: int, n2: int, precision: int):
    out = zm_pair_tuning()
    st = load().zm_tuning_get(n1, n2, precision, ctypes.byref(out))
    if st != ZM_OK:
        raise ZMError(st, "tuning_get")
    return int(out.targets_per_lane), int(out.source_splits)


def autotune(p: "Params", stream=None):
    """Time the candidate launch shapes for p's mesh size, store the fastest
    in the process-wide table; returns (targets_per_lane, splits, ms)."""
    import torch
    lib = load()
    nbytes = int(lib.zm_autotune_workspace_bytes(ctypes.byref(p.c())))
    if nbytes == 0:
        raise ZMError(ZM_ERR_INVALID_ARG, "invalid parameters")
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream() if stream is None else stream
    best = zm_pair_tuning()
    ms = ctypes.c_double()
    st = lib.zm_autotune(ctypes.byref(p.c()), ws.data_ptr(), nbytes, stream.cuda_stream,
                         ctypes.byref(best), ctypes.byref(ms))
    if st != ZM_OK:
        raise ZMError(st, "autotune")
    return int(best.targets_per_lane), int(best.source_splits), float(ms.value)


def _params_array(ps):
    arr = (zm_params * len(ps))()
    for i, p in enumerate(ps):
        arr[i] = p.c()
    return arr


def batch_autotune(ps, stream=None):
    """Choose the pair-kernel shape of every mesh size of a batch by timing
    the batched persistent sweep itself (zm_batch_autotune); the choices go
    into the process-wide table.  Returns ([(targets_per_lane, splits)] per
    member, ms of one batched pair sweep with them)."""
    import torch
    lib = load()
    arr = _params_array(ps)
    nbytes = int(lib.zm_batch_autotune_workspace_bytes(arr, len(ps)))
    if nbytes == 0:
        raise ZMError(ZM_ERR_INVALID_ARG, "invalid batch parameters")
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream() if stream is None else stream
    best = (zm_pair_tuning * len(ps))()
    ms = ctypes.c_double()
    st = lib.zm_batch_autotune(arr, len(ps), ws.data_ptr(), nbytes, stream.cuda_stream, best,
                               ctypes.byref(ms))
    if st != ZM_OK:
        raise ZMError(st, "batch autotune")
    return [(int(b.targets_per_lane), int(b.source_splits)) for b in best], float(ms.value)


def batch_workspace_bytes(ps) -> int:
    return int(load().zm_batch_workspace_bytes(_params_array(ps), len(ps)))


class Batch:
    """One zm_batch: many independent instances advanced together."""

    def __init__(self, ps, flags: int = 0, stream=None, device=None):
        import torch
        self.lib = load()
        self.params = list(ps)
        dev = torch.device("cuda", torch.cuda.current_device()) if device is None else device
        arr = _params_array(self.params)
        nbytes = int(self.lib.zm_batch_workspace_bytes(arr, len(self.params)))
        if nbytes == 0:
            raise ZMError(ZM_ERR_INVALID_ARG, "invalid batch parameters")
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        self.stream = torch.cuda.current_stream(dev) if stream is None else stream
        h = ctypes.c_void_p()
        with torch.cuda.device(dev):
            st = self.lib.zm_batch_create(ctypes.byref(h), arr, len(self.params), int(flags),
                                          self.workspace.data_ptr(), nbytes,
                                          self.stream.cuda_stream)
        if st != ZM_OK:
            raise ZMError(st, self.lib.zm_batch_last_error(None).decode())
        self.handle = h

    def _raise(self, st):
        if st != ZM_OK:
            raise ZMError(st, self.lib.zm_batch_last_error(self.handle).decode())

    def init_state(self, i: int, z, w):
        n = self.params[i].n
        _check_f64_planes(z, 3, n, "z"); _check_f64_planes(w, 2, n, "w")
        self._raise(self.lib.zm_batch_init_state(self.handle, int(i), _ptr(z), _ptr(w)))

    def get_state(self, i: int, z, w):
        n = self.params[i].n
        _check_f64_planes(z, 3, n, "z"); _check_f64_planes(w, 2, n, "w")
        self._raise(self.lib.zm_batch_get_state(self.handle, int(i), _ptr(z), _ptr(w)))

    def step(self, nsteps: int):
        self._raise(self.lib.zm_batch_step(self.handle, int(nsteps)))

    def info(self) -> zm_batch_info:
        out = zm_batch_info()
        self._raise(self.lib.zm_batch_get_info(self.handle, ctypes.byref(out)))
        return out

    def destroy(self):
        if getattr(self, "handle", None) is not None:
            st = self.lib.zm_batch_destroy(self.handle)
            self.handle = None
            if st != ZM_OK:
                raise ZMError(st, "batch destroy")

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def br_velocity_noalloc(p: Params, z, w, u, stream=None):
    """u = BR velocity of (z, w) through zm_br_velocity_noalloc: no context,
    no workspace, scratch in the library's static device array (calls that
    may overlap on one device race on it).  Enqueued on `stream` (default:
    the current torch stream)."""
    import torch
    lib = load()
    _check_f64_planes(z, 3, p.n, "z"); _check_f64_planes(w, 2, p.n, "w")
    _check_f64_planes(u, 3, p.n, "u")
    s = torch.cuda.current_stream(z.device) if stream is None else stream
    with torch.cuda.device(z.device):
        st = lib.zm_br_velocity_noalloc(ctypes.byref(p.c()), _ptr(z), _ptr(w), _ptr(u),
                                        s.cuda_stream)
    if st != ZM_OK:
        raise ZMError(st, lib.zm_last_error(None).decode())


def pool_request_bytes(p: Params) -> int:
    return int(load().zm_pool_request_bytes(ctypes.byref(p.c())))


class Pool:
    """One zm_pool: continuous batching of simulation requests."""

    def __init__(self, budget_bytes: int, flags: int = 0, stream=None, device=None):
        import torch
        self.lib = load()
        dev = torch.device("cuda", torch.cuda.current_device()) if device is None else device
        nbytes = int(self.lib.zm_pool_workspace_bytes(int(budget_bytes)))
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        self.stream = torch.cuda.current_stream(dev) if stream is None else stream
        self._inputs = {}          # id -> (z, w) kept alive until admitted
        self._points = {}          # id -> mesh points of the request (checks fetch buffers)
        h = ctypes.c_void_p()
        with torch.cuda.device(dev):
            st = self.lib.zm_pool_create(ctypes.byref(h), int(budget_bytes), int(flags),
                                         self.workspace.data_ptr(), nbytes, self.stream.cuda_stream)
        if st != ZM_OK:
            raise ZMError(st, self.lib.zm_pool_last_error(None).decode())
        self.handle = h
        self._rec = (zm_step_record * 4096)()

    def _raise(self, st):
        if st != ZM_OK:
            raise ZMError(st, self.lib.zm_pool_last_error(self.handle).decode())

    def submit(self, p: Params, z, w, steps: int) -> int:
        _check_f64_planes(z, 3, p.n, "z"); _check_f64_planes(w, 2, p.n, "w")
        rid = ctypes.c_int64()
        self._raise(self.lib.zm_pool_submit(self.handle, ctypes.byref(p.c()), _ptr(z), _ptr(w),
                                            int(steps), ctypes.byref(rid)))
        self._inputs[rid.value] = (z, w)
        self._points[rid.value] = p.n
        return rid.value

    def iterate(self):
        """One iteration; returns [(id, steps_done, state, iteration_ms)]."""
        n = ctypes.c_int32()
        self._raise(self.lib.zm_pool_iterate(self.handle, self._rec, len(self._rec), ctypes.byref(n)))
        out = [(r.id, r.steps_done, r.state, r.iteration_ms) for r in self._rec[:n.value]]
        for rid in list(self._inputs):
            if self.query(rid)[0] != ZM_REQ_QUEUED:
                del self._inputs[rid]
        return out

    def query(self, rid: int):
        st, done = ctypes.c_int32(), ctypes.c_int32()
        self._raise(self.lib.zm_pool_query(self.handle, int(rid), ctypes.byref(st), ctypes.byref(done)))
        return st.value, done.value

    def fetch(self, rid: int, z, w):
        n = self._points.get(int(rid))
        if n is None:
            raise ZMError(ZM_ERR_INVALID_ARG, f"request {rid} was not submitted through this pool "
                                               "or was already released")
        _check_f64_planes(z, 3, n, "z"); _check_f64_planes(w, 2, n, "w")
        self._raise(self.lib.zm_pool_fetch(self.handle, int(rid), _ptr(z), _ptr(w)))

    def release(self, rid: int):
        self._raise(self.lib.zm_pool_release(self.handle, int(rid)))
        self._points.pop(int(rid), None)

    def cancel(self, rid: int):
        self._raise(self.lib.zm_pool_cancel(self.handle, int(rid)))
        self._inputs.pop(rid, None)
        self._points.pop(int(rid), None)

    def stats(self) -> zm_pool_stats:
        out = zm_pool_stats()
        self._raise(self.lib.zm_pool_get_stats(self.handle, ctypes.byref(out)))
        return out

    def destroy(self):
        if getattr(self, "handle", None) is not None:
            st = self.lib.zm_pool_destroy(self.handle)
            self.handle = None
            if st != ZM_OK:
                raise ZMError(st, "pool destroy")

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass
