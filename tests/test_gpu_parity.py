"""GPU path (libzm.so through its C ABI) against the CPU oracle.

Floating-point bar: 1e-12 normwise relative error (max |gpu - oracle| /
max |oracle|) for the float64 path, on the same seeded inputs.  Sizes span
several target patches and source tiles with ragged tails; the full-size
workloads are checked on sampled targets the oracle evaluates one by one.
"""
import math

import numpy as np
import pytest

import oracle
import rocket_rig as rr
from zm_testutil import relerr, to_dev, to_host

pytestmark = pytest.mark.gpu

TOL64 = 1e-12


def params(n1, n2, **kw):
    import paper_2406_05490_amd as zm
    kw.setdefault("eps", 0.5 * 2.0 / n1)
    return zm.Params(n1, n2, **kw)


def oparams(p):
    return oracle.Problem(p.n1, p.n2, eps=p.eps, atwood=p.atwood, gravity=p.gravity, dt=p.dt,
                          nu=p.nu, images=p.image_layers, period1=p.period1, period2=p.period2)


def gpu_br(p, z, w, device):
    import paper_2406_05490_amd as zm
    import torch
    ctx = zm.Context(p)
    zd, wd = to_dev(z, device), to_dev(w, device)
    ud = torch.empty(3 * p.n, dtype=torch.float64, device=device)
    ctx.br_velocity(zd, wd, ud)
    torch.cuda.synchronize()
    return to_host(ud, (3, p.n)), ctx


@pytest.mark.parametrize("n1,n2,seed", [
    (8, 8, 0), (64, 64, 1), (40, 24, 2), (33, 27, 3), (48, 96, 4), (17, 130, 5), (96, 40, 6),
    (9, 8, 7), (300, 12, 8), (12, 520, 9), (160, 24, 10), (64, 200, 11),
])
def test_br_velocity_matches_oracle(gpu, n1, n2, seed):
    p = params(n1, n2)
    z, w = rr.random_state(n1, n2, seed=seed, height=0.1)
    u, _ = gpu_br(p, z, w, gpu)
    ref = oracle.br_velocity(oparams(p), z, w)
    assert relerr(u, ref) < TOL64


@pytest.mark.parametrize("K", [1, 2])
def test_br_velocity_image_layers(gpu, K):
    p = params(16, 12, image_layers=K)
    z, w = rr.random_state(16, 12, seed=11, height=0.1)
    u, _ = gpu_br(p, z, w, gpu)
    assert relerr(u, oracle.br_velocity(oparams(p), z, w)) < TOL64


def test_br_velocity_nonsquare_period(gpu):
    p = params(24, 16, period1=3.0, period2=1.5, eps=0.05)
    z, w = rr.random_state(24, 16, seed=12, height=0.1)
    A1 = -1.5 + np.arange(24) * (3.0 / 24); A2 = -0.75 + np.arange(16) * (1.5 / 16)
    X, Y = np.meshgrid(A1, A2)
    z[0] = X.ravel(); z[1] = Y.ravel()
    u, _ = gpu_br(p, z, w, gpu)
    assert relerr(u, oracle.br_velocity(oparams(p), z, w)) < TOL64


def test_flat_sheet_eigenvalue_on_gpu(gpu):
    """The flat-sheet closed-form check, run on the GPU: tangential velocity
    exactly 0 and u3 an eigenvector of the cos mode."""
    n = 64
    p = params(n, n)
    z, _ = rr.flat_state(n, n)
    A1, A2 = rr.grid(n, n)
    k1, k2 = math.pi, 2 * math.pi
    mu = np.cos(k1 * A1 + k2 * A2).ravel()
    s = np.sin(k1 * A1 + k2 * A2).ravel()
    w = np.stack([-k1 * s, -k2 * s])
    u, _ = gpu_br(p, z, w, gpu)
    assert np.all(u[0] == 0.0) and np.all(u[1] == 0.0)
    lam = float(u[2] @ mu / (mu @ mu))
    assert np.max(np.abs(u[2] - lam * mu)) < 1e-12 * abs(lam)
    ref = oracle.br_velocity(oparams(p), z, w)
    assert relerr(u, ref) < TOL64


def test_rest_state_exact(gpu):
    import paper_2406_05490_amd as zm
    import torch
    n = 32
    p = params(n, n)
    z, w = rr.flat_state(n, n)
    u, _ = gpu_br(p, z, w, gpu)
    assert np.all(u == 0.0)
    ctx = zm.Context(p)
    zd, wd = to_dev(z, gpu), to_dev(w, gpu)
    ctx.init_state(zd, wd)
    ctx.step(3)
    z1 = torch.empty_like(zd); w1 = torch.empty_like(wd)
    ctx.get_state(z1, w1)
    torch.cuda.synchronize()
    z1 = to_host(z1, (3, n * n)); w1 = to_host(w1, (2, n * n))
    assert np.all(z1[2] == 0.0) and np.all(w1 == 0.0)
    assert np.max(np.abs(z1[:2] - z[:2])) <= 6 * np.finfo(np.float64).eps


def test_symmetries_bitwise_on_gpu(gpu):
    n1, n2 = 48, 40
    p = params(n1, n2)
    z, w = rr.random_state(n1, n2, seed=13, height=0.1)
    u, _ = gpu_br(p, z, w, gpu)
    um, _ = gpu_br(p, z, -w, gpu)
    assert np.array_equal(um, -u)
    zm_ = z.copy(); zm_[2] = -zm_[2]
    uv, _ = gpu_br(p, zm_, w, gpu)
    assert np.array_equal(uv[:2], -u[:2]) and np.array_equal(uv[2], u[2])


def test_periodic_translation_on_gpu(gpu):
    n1, n2 = 32, 24
    p = params(n1, n2)
    z, w = rr.random_state(n1, n2, seed=14, height=0.1)
    u, _ = gpu_br(p, z, w, gpu)
    Z = z.reshape(3, n2, n1); W = w.reshape(2, n2, n1)
    s = 7
    idx = (np.arange(n1) + s) % n1
    wraps = (np.arange(n1) + s) // n1
    Zr = Z[:, :, idx].copy(); Wr = W[:, :, idx].copy()
    Zr[0] = Zr[0] + wraps[None, :] * 2.0
    ur, _ = gpu_br(p, Zr.reshape(3, -1), Wr.reshape(2, -1), gpu)
    assert relerr(ur.reshape(3, n2, n1), u.reshape(3, n2, n1)[:, :, idx]) < 1e-13


def test_repeat_is_bitwise_deterministic(gpu):
    n = 64
    p = params(n, n)
    z, w = rr.random_state(n, n, seed=15, height=0.1)
    a, _ = gpu_br(p, z, w, gpu)
    b, _ = gpu_br(p, z, w, gpu)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("n1,n2,nu", [(64, 64, 0.0), (36, 20, 0.0), (24, 30, 1e-3)])
def test_rhs_matches_oracle(gpu, n1, n2, nu):
    import paper_2406_05490_amd as zm
    import torch
    p = params(n1, n2, atwood=0.7, gravity=1.3, nu=nu)
    z, w = rr.random_state(n1, n2, seed=16, height=0.1)
    ctx = zm.Context(p)
    zd, wd = to_dev(z, gpu), to_dev(w, gpu)
    zt = torch.empty_like(zd); wt = torch.empty_like(wd)
    ctx.rhs(zd, wd, zt, wt)
    torch.cuda.synchronize()
    rz, rw = oracle.rhs(oparams(p), z, w)
    assert relerr(to_host(zt, (3, -1)), rz) < TOL64
    assert relerr(to_host(wt, (2, -1)), rw) < TOL64


def run_gpu_steps(p, z, w, nsteps, device, chunks=1):
    import paper_2406_05490_amd as zm
    import torch
    ctx = zm.Context(p)
    zd, wd = to_dev(z, device), to_dev(w, device)
    ctx.init_state(zd, wd)
    for _ in range(chunks):
        ctx.step(nsteps // chunks)
    z1 = torch.empty_like(zd); w1 = torch.empty_like(wd)
    ctx.get_state(z1, w1)
    torch.cuda.synchronize()
    return to_host(z1, (3, p.n)), to_host(w1, (2, p.n))


def test_periodic64_single_mode_trajectory(gpu):
    """64 x 64 single mode + 1e-4 noise (seed 0), A = 0.5, g = 1,
    eps = h/2, dt = 1e-3, 10 RK3 steps: full trajectory against the oracle."""
    wl = rr.WORKLOADS["periodic64_single_fp64"]
    p = params(wl.n1, wl.n2, atwood=wl.atwood, gravity=wl.gravity, dt=wl.dt, eps=wl.eps)
    z, w = wl.state()
    zg, wg = run_gpu_steps(p, z, w, wl.steps, gpu)
    zr, wr = oracle.rk3(oparams(p), z, w, wl.steps)
    assert relerr(zg, zr) < TOL64
    assert relerr(wg, wr) < TOL64
    assert relerr(zg - z, zr - z) < 1e-9          # the motion itself, not just the state


def test_checkpoint_resume_bitwise(gpu):
    n = 32
    p = params(n, n, atwood=0.5, dt=2e-3)
    z, w = rr.single_mode(n, n, 0.05, noise=1e-4, seed=3)
    a = run_gpu_steps(p, z, w, 6, gpu)
    b = run_gpu_steps(p, z, w, 6, gpu, chunks=3)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_periodic256_multimode_sampled(gpu):
    """256 x 256, 8 modes + noise (seed 1), 50 steps on the GPU; the oracle
    evaluates F at the GPU state after steps 0, 1, 10 and 50 on 256 seeded
    targets (BR at the targets and their stencil neighbours)."""
    import paper_2406_05490_amd as zm
    import torch
    wl = rr.WORKLOADS["periodic256_multimode8_fp64"]
    p = params(wl.n1, wl.n2, atwood=wl.atwood, gravity=wl.gravity, dt=wl.dt, eps=wl.eps)
    z, w = wl.state()
    ctx = zm.Context(p)
    zd, wd = to_dev(z, gpu), to_dev(w, gpu)
    ctx.init_state(zd, wd)
    tg = rr.sample_targets(p.n, 256, seed=wl.seed)
    done = 0
    for mark in (0, 1, 10, 50):
        ctx.step(mark - done)
        done = mark
        zs = torch.empty_like(zd); ws = torch.empty_like(wd)
        ctx.get_state(zs, ws)
        zt = torch.empty_like(zd); wt = torch.empty_like(wd)
        ctx.rhs(zs, ws, zt, wt)
        torch.cuda.synchronize()
        zh, wh = to_host(zs, (3, p.n)), to_host(ws, (2, p.n))
        rz, rw = oracle.rhs_sampled(oparams(p), zh, wh, tg)
        gz, gw = to_host(zt, (3, p.n))[:, tg], to_host(wt, (2, p.n))[:, tg]
        assert relerr(gz, rz) < TOL64, f"z_t after {mark} steps"
        assert relerr(gw, rw) < TOL64, f"w_t after {mark} steps"


def test_periodic1024_br_sampled(gpu):
    """The 1M-point sweep (1024 x 1024, 16 modes, synthetic vorticity),
    float64, against the oracle on 64 seeded targets."""
    wl = rr.WORKLOADS["periodic1024_multimode16_fp32"]
    p = params(wl.n1, wl.n2, atwood=wl.atwood, eps=wl.eps)
    z, _ = wl.state()
    w = rr.synthetic_vorticity(wl.n1, wl.n2, seed=wl.seed)
    u, _ = gpu_br(p, z, w, gpu)
    tg = rr.sample_targets(p.n, 64, seed=wl.seed)
    ref = oracle.br_velocity(oparams(p), z, w, targets=tg)
    assert relerr(u[:, tg], ref) < TOL64


def test_launch_info(gpu):
    import paper_2406_05490_amd as zm
    ctx = zm.Context(params(256, 256))
    info = ctx.launch_info()
    assert info.pairs_per_eval == 65536 ** 2
    assert info.workgroups >= 256 and info.threads_per_group == 256


@pytest.mark.parametrize("n1,n2", [(48, 40), (40, 33), (33, 40)])
def test_eager_graph_profiled_steps_agree(gpu, n1, n2):
    """Meshes with tie columns or rows (an even side): eager steps,
    graph-replayed steps and profiled steps (timing events around every
    launch) give the same state bit for bit, and match the oracle."""
    import paper_2406_05490_amd as zm
    import torch
    z, w = rr.random_state(n1, n2, seed=11, height=0.1)
    out = []
    for flags, prof in ((0, False), (zm.ZM_FLAG_GRAPH, False), (0, True)):
        p = params(n1, n2, atwood=0.5, dt=2e-3, flags=flags)
        ctx = zm.Context(p)
        zd, wd = to_dev(z, gpu), to_dev(w, gpu)
        ctx.init_state(zd, wd)
        ctx.profile_enable(prof)
        ctx.step(2)
        ctx.step(2)
        z1 = torch.empty_like(zd); w1 = torch.empty_like(wd)
        ctx.get_state(z1, w1)
        torch.cuda.synchronize()
        if prof:
            assert ctx.profile_read()["ties"][0] == 12
        out.append((to_host(z1, (3, p.n)), to_host(w1, (2, p.n))))
    for zs, ws in out[1:]:
        assert np.array_equal(zs, out[0][0]) and np.array_equal(ws, out[0][1])
    zr, wr = oracle.rk3(oparams(params(n1, n2, atwood=0.5, dt=2e-3)), z, w, 4)
    assert relerr(out[0][0], zr) < TOL64 and relerr(out[0][1], wr) < TOL64


def test_profile_counts_launches(gpu):
    import paper_2406_05490_amd as zm
    import torch
    n = 32
    p = params(n, n)
    z, w = rr.single_mode(n, n, 0.05)
    ctx = zm.Context(p)
    ctx.init_state(to_dev(z, gpu), to_dev(w, gpu))
    ctx.profile_enable(True)
    ctx.step(2)
    st = ctx.profile_read()
    assert st["pairs"][0] == 6 and st["update"][0] == 6 and st["ties"][0] == 6
    assert st["pairs"][1] > 0.0
    ctx.profile_enable(False)
    ctx.step(1)
    torch.cuda.synchronize()
    assert ctx.profile_read()["pairs"][0] == 0


# --------------------------------------------------------------------------
# error paths (forced from the host; every kernel still exits normally)
# --------------------------------------------------------------------------

def test_nonfinite_state_is_reported(gpu):
    import paper_2406_05490_amd as zm
    n = 16
    p = params(n, n, flags=zm.ZM_FLAG_CHECK_FINITE)
    z, w = rr.single_mode(n, n, 0.05)
    z[2, 37] = np.nan
    ctx = zm.Context(p)
    ctx.init_state(to_dev(z, gpu), to_dev(w, gpu))
    with pytest.raises(zm.ZMError) as e:
        ctx.step(1)
    assert e.value.status == zm.ZM_ERR_NONFINITE
    # a clean state passes the same check
    ctx2 = zm.Context(p)
    z2, w2 = rr.single_mode(n, n, 0.05)
    ctx2.init_state(to_dev(z2, gpu), to_dev(w2, gpu))
    ctx2.step(2)


def test_bad_pointers_rejected(gpu):
    import ctypes
    import paper_2406_05490_amd as zm
    import torch
    n = 16
    p = params(n, n)
    ctx = zm.Context(p)
    z = torch.zeros(3 * n * n + 8, dtype=torch.float64, device=gpu)
    w = torch.zeros(2 * n * n, dtype=torch.float64, device=gpu)
    lib = zm.load()
    # misaligned
    st = lib.zm_br_velocity(ctx.handle, z.data_ptr() + 8, w.data_ptr(), z.data_ptr())
    assert st == zm.ZM_ERR_INVALID_ARG
    # output overlapping an input
    st = lib.zm_br_velocity(ctx.handle, z.data_ptr(), w.data_ptr(), w.data_ptr())
    assert st == zm.ZM_ERR_INVALID_ARG
    assert "overlap" in lib.zm_last_error(ctx.handle).decode()
    assert lib.zm_step(ctx.handle, -1) == zm.ZM_ERR_INVALID_ARG
    with pytest.raises(ValueError):
        ctx.br_velocity(z[:3 * n * n].float(), w, z[:3 * n * n])
