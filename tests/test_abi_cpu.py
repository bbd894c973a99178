"""The C ABI library loads, exports what include/zm.h declares, and rejects
bad arguments on the host (no GPU needed: these checks run before any HIP
call)."""
import ctypes
import os
import re

import pytest

import paper_2406_05490_amd as zm
from paper_2406_05490_amd import _zm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "zm.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return re.findall(r"\b(zm_[a-z0-9_]+)\s*\(", src)


def test_header_declares_binding_exports():
    assert tuple(declared_functions()) == _zm.EXPORTS


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(zm.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_abi_version_and_status_strings():
    lib = zm.load()
    assert lib.zm_abi_version() == 5
    assert zm.status_string(zm.ZM_OK) == "ok"
    for st in (zm.ZM_ERR_INVALID_ARG, zm.ZM_ERR_UNSUPPORTED, zm.ZM_ERR_WORKSPACE,
               zm.ZM_ERR_HIP, zm.ZM_ERR_NONFINITE, zm.ZM_ERR_CAPACITY):
        assert zm.status_string(st) not in ("ok", "unknown status")
    assert zm.status_string(12345) == "unknown status"


def test_struct_layout_matches_header():
    # n1 n2 (8) + 7 doubles (56) + 4 int32 (16) + cutoff (8) + 2 int32 (8)
    assert ctypes.sizeof(_zm.zm_params) == 96
    assert ctypes.sizeof(_zm.zm_cutoff_info) == 40
    assert ctypes.sizeof(_zm.zm_launch_info) == 32
    assert ctypes.sizeof(_zm.zm_kernel_stats) == 16


@pytest.mark.parametrize("bad", [
    dict(n1=7), dict(n2=4), dict(n1=20000), dict(eps=0.0), dict(eps=-1.0),
    dict(eps=float("nan")), dict(dt=0.0), dict(nu=-1.0), dict(period1=0.0),
    dict(atwood=float("inf")), dict(precision=7), dict(image_layers=-1),
    dict(image_layers=17), dict(flags=0x80), dict(cutoff=-0.1), dict(cutoff=float("nan")),
    dict(cutoff=0.95), dict(cutoff=0.3, image_layers=1), dict(cutoff=0.3, precision=1),
    dict(model=1, cutoff=0.3), dict(model=1, image_layers=1),
    dict(model=1, precision=1), dict(model=1, n1=24),
    dict(boundary=2), dict(boundary=1, model=1), dict(boundary=1, image_layers=1),
    dict(boundary=1, cutoff=-0.5), dict(model=3), dict(model=2, boundary=1),
])
def test_workspace_bytes_rejects_invalid(bad):
    kw = dict(n1=16, n2=16, eps=1 / 16)
    kw.update(bad)
    assert zm.workspace_bytes(zm.Params(**kw)) == 0


def test_cutoff_workspace_and_status():
    """A cutoff context needs extra workspace (cell list, sorted copies); an
    FP32 cutoff request is a valid one this build does not provide."""
    a = zm.workspace_bytes(zm.Params(64, 64, eps=1 / 64))
    b = zm.workspace_bytes(zm.Params(64, 64, eps=1 / 64, cutoff=0.3))
    assert 0 < a < b and b % 256 == 0
    st, _, msg = _create(zm.Params(64, 64, eps=1 / 64, cutoff=0.3, precision=1), None, 0)
    assert st == zm.ZM_ERR_UNSUPPORTED and "FP64" in msg
    st, _, msg = _create(zm.Params(64, 64, eps=1 / 64, cutoff=0.95), None, 0)
    assert st == zm.ZM_ERR_INVALID_ARG and "cutoff" in msg


def test_free_sheet_cutoff_takes_any_radius():
    """A free sheet has no images, so the cutoff is not bounded by the period."""
    a = zm.workspace_bytes(zm.Params(64, 64, eps=1 / 64, boundary=zm.ZM_BOUNDARY_FREE, cutoff=0.3))
    b = zm.workspace_bytes(zm.Params(64, 64, eps=1 / 64, boundary=zm.ZM_BOUNDARY_FREE, cutoff=5.0))
    assert a > 0 and b > 0
    assert zm.workspace_bytes(zm.Params(64, 64, eps=1 / 64, cutoff=5.0)) == 0


def test_fp32_refused_on_very_anisotropic_meshes():
    """The FP32 pair form needs pair patches within 128 finest mesh spacings;
    8192 x 8 on a square period spans thousands.  FP64 serves the same mesh;
    square meshes always pass."""
    for n1, n2 in ((8192, 8), (8, 8192), (4096, 16)):
        p32 = zm.Params(n1, n2, eps=1e-3, precision=zm.ZM_FP32_PAIRS)
        assert zm.workspace_bytes(p32) == 0
        st, _, msg = _create(p32, None, 0)
        assert st == zm.ZM_ERR_UNSUPPORTED and "anisotropic" in msg
        assert zm.workspace_bytes(zm.Params(n1, n2, eps=1e-3)) > 0
        assert zm.batch_workspace_bytes([p32]) == 0
        assert zm.pool_request_bytes(p32) == 0
    for n in (8, 12, 33, 64, 256, 1024, 8192):
        assert zm.workspace_bytes(zm.Params(n, n, eps=1.0 / n, precision=zm.ZM_FP32_PAIRS)) > 0
    assert zm.workspace_bytes(zm.Params(1024, 256, eps=1e-3, precision=zm.ZM_FP32_PAIRS)) > 0


def test_medium_order_workspace_and_status():
    """Medium order: the BR workspace plus the FFT buffers; power-of-two sides."""
    hi = zm.workspace_bytes(zm.Params(64, 64, eps=1 / 64))
    me = zm.workspace_bytes(zm.Params(64, 64, eps=1 / 64, model=zm.ZM_MODEL_MEDIUM))
    assert 0 < hi < me and me % 256 == 0
    assert zm.workspace_bytes(zm.Params(64, 64, eps=1 / 64, model=zm.ZM_MODEL_MEDIUM, cutoff=0.3)) > me
    assert zm.workspace_bytes(zm.Params(64, 64, eps=1 / 64, model=zm.ZM_MODEL_MEDIUM,
                                        precision=zm.ZM_FP32_PAIRS)) > 0
    assert zm.workspace_bytes(zm.Params(48, 64, eps=1 / 48, model=zm.ZM_MODEL_MEDIUM)) == 0
    st, _, msg = _create(zm.Params(48, 64, eps=1 / 48, model=zm.ZM_MODEL_MEDIUM), None, 0)
    assert st == zm.ZM_ERR_UNSUPPORTED and "powers of two" in msg
    p = zm.Params(32, 32, eps=1 / 32, model=zm.ZM_MODEL_MEDIUM)
    assert zm.batch_workspace_bytes([p]) == 0
    assert zm.pool_request_bytes(p) == 0


def test_low_order_workspace_and_status():
    a = zm.workspace_bytes(zm.Params(64, 64, eps=1 / 64))
    b = zm.workspace_bytes(zm.Params(64, 64, eps=1 / 64, model=zm.ZM_MODEL_LOW))
    assert 0 < a < b and b % 256 == 0
    st, _, msg = _create(zm.Params(48, 64, eps=1 / 48, model=zm.ZM_MODEL_LOW), None, 0)
    assert st == zm.ZM_ERR_UNSUPPORTED and "powers of two" in msg
    st, _, msg = _create(zm.Params(64, 64, eps=1 / 64, model=zm.ZM_MODEL_LOW, cutoff=0.3), None, 0)
    assert st == zm.ZM_ERR_INVALID_ARG
    p = zm.Params(32, 32, eps=1 / 32, model=zm.ZM_MODEL_LOW)
    assert zm.batch_workspace_bytes([p]) == 0
    assert zm.pool_request_bytes(p) == 0


def test_cutoff_refused_by_batches_and_pools():
    p = zm.Params(32, 32, eps=1 / 32, cutoff=0.3)
    assert zm.batch_workspace_bytes([p]) == 0
    assert zm.pool_request_bytes(p) == 0


def test_workspace_bytes_grows_with_mesh():
    a = zm.workspace_bytes(zm.Params(16, 16, eps=1 / 16))
    b = zm.workspace_bytes(zm.Params(64, 64, eps=1 / 64))
    assert 0 < a < b
    assert a % 256 == 0 and b % 256 == 0


def _create(p, ws, nbytes):
    lib = zm.load()
    h = ctypes.c_void_p(1234)
    st = lib.zm_create(ctypes.byref(h), ctypes.byref(p.c()), ws, nbytes, None)
    return st, h, lib.zm_last_error(None).decode()


def test_create_rejects_bad_params_without_touching_device():
    st, h, msg = _create(zm.Params(4, 16, eps=0.1), 256, 1 << 20)
    assert st == zm.ZM_ERR_INVALID_ARG and h.value is None and "n1" in msg


def test_create_rejects_missing_or_small_workspace():
    p = zm.Params(16, 16, eps=1 / 16)
    need = zm.workspace_bytes(p)
    st, h, msg = _create(p, None, need)
    assert st == zm.ZM_ERR_WORKSPACE and h.value is None
    st, h, msg = _create(p, 256 * 3 + 8, need)          # misaligned
    assert st == zm.ZM_ERR_WORKSPACE
    st, h, msg = _create(p, 4096, need - 1)             # too small
    assert st == zm.ZM_ERR_WORKSPACE and "smaller" in msg


def test_null_context_calls_are_rejected():
    lib = zm.load()
    assert lib.zm_step(None, 1) == zm.ZM_ERR_INVALID_ARG
    assert lib.zm_init_state(None, None, None) == zm.ZM_ERR_INVALID_ARG
    assert lib.zm_br_velocity(None, None, None, None) == zm.ZM_ERR_INVALID_ARG
    assert lib.zm_destroy(None) == zm.ZM_OK


def test_batch_workspace_validation():
    ok = [zm.Params(16, 16, eps=1 / 16), zm.Params(32, 24, eps=1 / 32, precision=zm.ZM_FP32_PAIRS)]
    assert zm.batch_workspace_bytes(ok) > zm.workspace_bytes(ok[0]) + zm.workspace_bytes(ok[1])
    assert zm.batch_workspace_bytes(ok + [zm.Params(4, 16, eps=1.0)]) == 0
    assert zm.batch_workspace_bytes([zm.Params(16, 16, eps=1 / 16, flags=1)]) == 0
    lib = zm.load()
    assert lib.zm_batch_workspace_bytes(None, 1) == 0


def test_tuning_table_host_side():
    """The shape table is host state: set, read back, clear, reject bad."""
    d = zm.tuning_get(96, 80, zm.ZM_FP64)
    assert d[0] in (1, 2, 4) and 1 <= d[1] <= 80
    zm.tuning_set(96, 80, zm.ZM_FP64, 2, 10)
    assert zm.tuning_get(96, 80, zm.ZM_FP64) == (2, 10)
    zm.tuning_set(96, 80, zm.ZM_FP64, 4, 1000)           # clamped to n2 rows
    assert zm.tuning_get(96, 80, zm.ZM_FP64) == (4, 80)
    zm.tuning_set(96, 80, zm.ZM_FP64)                     # remove
    assert zm.tuning_get(96, 80, zm.ZM_FP64) == d
    with pytest.raises(zm.ZMError):
        zm.tuning_set(96, 80, zm.ZM_FP64, 3, 10)
    with pytest.raises(zm.ZMError):
        zm.tuning_set(4, 80, zm.ZM_FP64, 1, 1)
    lib = zm.load()
    assert lib.zm_autotune_workspace_bytes(ctypes.byref(zm.Params(64, 64, eps=1 / 64).c())) > 0


def test_default_shapes_large_fp32_meshes():
    """Untuned defaults: FP32 from 2^20 points up takes about 32768
    workgroups (source splits), so partial sums stay near 400 MB; smaller
    FP32 meshes (batch and serving sizes) and FP64 keep the >= 2048-workgroup
    rule with twice its splits."""
    assert zm.tuning_get(1024, 1024, zm.ZM_FP32_PAIRS) == (2, 16)     # 2048 patches
    assert zm.tuning_get(2048, 2048, zm.ZM_FP32_PAIRS) == (2, 4)      # 8192 patches
    assert zm.tuning_get(512, 512, zm.ZM_FP32_PAIRS) == (2, 8)
    assert zm.tuning_get(1024, 1024, zm.ZM_FP64) == (4, 4)
    p = zm.Params(1024, 1024, eps=1 / 1024, precision=zm.ZM_FP32_PAIRS)
    assert zm.workspace_bytes(p) > 16 * 3 * 1024 * 1024 * 8
    # the autotuner's candidates include the default, so its workspace holds it
    assert zm.load().zm_autotune_workspace_bytes(ctypes.byref(p.c())) >= 16 * 3 * 1024 * 1024 * 8


def test_pool_host_side_validation():
    p = zm.Params(64, 64, eps=1 / 64)
    rb = zm.pool_request_bytes(p)
    assert rb >= zm.workspace_bytes(p) - 256 and rb % 256 == 0
    assert zm.pool_request_bytes(zm.Params(4, 64, eps=1.0)) == 0
    assert zm.pool_request_bytes(zm.Params(64, 64, eps=1 / 64, flags=1)) == 0
    lib = zm.load()
    assert lib.zm_pool_workspace_bytes(1 << 30) > (1 << 30)
    h = ctypes.c_void_p(5)
    assert lib.zm_pool_create(ctypes.byref(h), 0, 0, 4096, 1 << 40, None) == zm.ZM_ERR_INVALID_ARG
    assert h.value is None
    assert lib.zm_pool_create(ctypes.byref(h), 1 << 20, 0, 4096, 1 << 10, None) == zm.ZM_ERR_WORKSPACE
    assert lib.zm_pool_create(ctypes.byref(h), 1 << 20, 0x40, 4096, 1 << 40, None) == zm.ZM_ERR_INVALID_ARG


def test_noalloc_host_side_validation():
    """zm_br_velocity_noalloc checks its arguments and its scratch limit on
    the host before any HIP call (fake, far-apart aligned addresses; nothing
    is launched)."""
    lib = zm.load()
    z, w, u = 1 << 40, 2 << 40, 3 << 40

    def call(p, zz=z, ww=w, uu=u):
        st = lib.zm_br_velocity_noalloc(ctypes.byref(p.c()), zz, ww, uu, None)
        return st, lib.zm_last_error(None).decode()

    st, msg = call(zm.Params(4, 16, eps=0.1))
    assert st == zm.ZM_ERR_INVALID_ARG and "n1" in msg
    st, msg = call(zm.Params(64, 64, eps=1 / 64, cutoff=0.2))
    assert st == zm.ZM_ERR_UNSUPPORTED and "exact" in msg
    st, msg = call(zm.Params(64, 64, eps=1 / 64, model=zm.ZM_MODEL_LOW))
    assert st == zm.ZM_ERR_UNSUPPORTED
    st, msg = call(zm.Params(64, 64, eps=1 / 64), zz=None)
    assert st == zm.ZM_ERR_INVALID_ARG and "aligned" in msg
    st, msg = call(zm.Params(64, 64, eps=1 / 64), uu=z + 8 * 256)
    assert st == zm.ZM_ERR_INVALID_ARG and "overlaps" in msg
    # even sides: 80 B per point before any partial sums -> 1024^2 cannot fit
    st, msg = call(zm.Params(1024, 1024, eps=1 / 1024))
    assert st == zm.ZM_ERR_CAPACITY and "scratch" in msg
    assert zm.NOALLOC_SCRATCH_BYTES == 64 * 1024 * 1024
