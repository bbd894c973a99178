"""FP32-interaction form (pair terms in float32 with tile-relative
coordinates, per-target sums in float64, state and RK3 in float64) against
the float64 oracle and the float64 GPU path.  Bar: 1e-5 normwise."""
import numpy as np
import pytest

import oracle
import rocket_rig as rr
from zm_testutil import relerr, to_dev, to_host

pytestmark = pytest.mark.gpu

TOL32 = 1e-5


def params(n1, n2, precision, **kw):
    import paper_2406_05490_amd as zm
    kw.setdefault("eps", 0.5 * 2.0 / n1)
    return zm.Params(n1, n2, precision=precision, **kw)


def gpu_br(p, z, w, device):
    import paper_2406_05490_amd as zm
    import torch
    ctx = zm.Context(p)
    zd, wd = to_dev(z, device), to_dev(w, device)
    ud = torch.empty(3 * p.n, dtype=torch.float64, device=device)
    ctx.br_velocity(zd, wd, ud)
    torch.cuda.synchronize()
    return to_host(ud, (3, p.n))


@pytest.mark.parametrize("n1,n2,seed", [(8, 8, 0), (64, 64, 1), (40, 24, 2), (33, 27, 3),
                                        (96, 40, 4), (17, 130, 5), (128, 128, 6)])
def test_fp32_br_matches_oracle(gpu, n1, n2, seed):
    import paper_2406_05490_amd as zm
    z, w = rr.random_state(n1, n2, seed=seed, height=0.1)
    p = params(n1, n2, zm.ZM_FP32_PAIRS)
    u = gpu_br(p, z, w, gpu)
    ref = oracle.br_velocity(oracle.Problem(n1, n2, eps=p.eps), z, w)
    assert relerr(u, ref) < TOL32


def test_fp32_image_layers(gpu):
    import paper_2406_05490_amd as zm
    z, w = rr.random_state(16, 12, seed=7, height=0.1)
    p = params(16, 12, zm.ZM_FP32_PAIRS, image_layers=1)
    u = gpu_br(p, z, w, gpu)
    ref = oracle.br_velocity(oracle.Problem(16, 12, eps=p.eps, images=1), z, w)
    assert relerr(u, ref) < TOL32


def test_fp32_rest_and_flat_sheet(gpu):
    import math
    import paper_2406_05490_amd as zm
    n = 64
    z, w0 = rr.flat_state(n, n)
    p = params(n, n, zm.ZM_FP32_PAIRS)
    assert np.all(gpu_br(p, z, w0, gpu) == 0.0)
    A1, A2 = rr.grid(n, n)
    s = np.sin(math.pi * A1 + 2 * math.pi * A2).ravel()
    w = np.stack([-math.pi * s, -2 * math.pi * s])
    u = gpu_br(p, z, w, gpu)
    assert np.all(u[0] == 0.0) and np.all(u[1] == 0.0)
    ref = oracle.br_velocity(oracle.Problem(n, n, eps=p.eps), z, w)
    assert relerr(u, ref) < TOL32


def test_fp32_1m_point_sweep(gpu):
    """1024 x 1024 (16 modes, synthetic vorticity): FP32 form against the FP64
    GPU path on all targets and the oracle on 64 seeded targets."""
    import paper_2406_05490_amd as zm
    wl = rr.WORKLOADS["periodic1024_multimode16_fp32"]
    z, _ = wl.state()
    w = rr.synthetic_vorticity(wl.n1, wl.n2, seed=wl.seed)
    u32 = gpu_br(params(wl.n1, wl.n2, zm.ZM_FP32_PAIRS, eps=wl.eps), z, w, gpu)
    u64 = gpu_br(params(wl.n1, wl.n2, zm.ZM_FP64, eps=wl.eps), z, w, gpu)
    assert relerr(u32, u64) < TOL32
    tg = rr.sample_targets(wl.n, 64, seed=wl.seed)
    ref = oracle.br_velocity(oracle.Problem(wl.n1, wl.n2, eps=wl.eps), z, w, targets=tg)
    assert relerr(u32[:, tg], ref) < TOL32
    assert relerr(u64[:, tg], ref) < 1e-12


def test_fp32_steps_track_fp64(gpu):
    """The 1024 x 1024 precision workload (A = 0.9, 5 RK3 steps): the FP32
    form's motion z - z0 and vorticity agree with the FP64 path."""
    import paper_2406_05490_amd as zm
    import torch
    wl = rr.WORKLOADS["periodic1024_multimode16_fp32"]
    z, w = wl.state()
    out = {}
    for prec in (zm.ZM_FP32_PAIRS, zm.ZM_FP64):
        p = params(wl.n1, wl.n2, prec, eps=wl.eps, atwood=wl.atwood, gravity=wl.gravity, dt=wl.dt)
        ctx = zm.Context(p)
        zd, wd = to_dev(z, gpu), to_dev(w, gpu)
        ctx.init_state(zd, wd)
        ctx.step(wl.steps)
        z1 = torch.empty_like(zd); w1 = torch.empty_like(wd)
        ctx.get_state(z1, w1)
        torch.cuda.synchronize()
        out[prec] = (to_host(z1, (3, -1)), to_host(w1, (2, -1)))
        del ctx
    (z32, w32), (z64, w64) = out[zm.ZM_FP32_PAIRS], out[zm.ZM_FP64]
    assert relerr(z32 - z, z64 - z) < TOL32
    assert relerr(w32, w64) < TOL32


def test_fp32_deterministic(gpu):
    import paper_2406_05490_amd as zm
    z, w = rr.random_state(64, 48, seed=9, height=0.1)
    p = params(64, 48, zm.ZM_FP32_PAIRS)
    assert np.array_equal(gpu_br(p, z, w, gpu), gpu_br(p, z, w, gpu))


def folded_state(n1, n2, depth=1.5, height=0.02, seed=9):
    """A sheet folded over itself along axis 2: z2 = a2 + depth/pi sin(pi a2)
    runs forward, back and forward over one period (depth > 1), so rows far
    apart in index lie a fraction of a spacing apart in space (0.09 spacings
    at 32 x 128) -- the situation of a rolled-up interface."""
    import math
    A1, A2 = rr.grid(n1, n2)
    z = np.stack([A1, A2 + (depth / math.pi) * np.sin(math.pi * A2),
                  height * np.cos(math.pi * A2)]).reshape(3, -1)
    w = rr.synthetic_vorticity(n1, n2, seed=seed)
    return z, w


@pytest.mark.parametrize("n1,n2", [(64, 128), (64, 96), (48, 160)])
def test_folded_sheet_matches_oracle_in_both_forms(gpu, n1, n2):
    """The expanded |r|^2 of the factored far form is only accurate for
    sources physically far from the patch; on a folded sheet many sources
    far in index are close in space, and both pair forms must still meet
    their bars (FP64 1e-12, FP32 1e-5)."""
    import paper_2406_05490_amd as zm
    z, w = folded_state(n1, n2)
    ref = oracle.br_velocity(oracle.Problem(n1, n2, eps=0.5 * 2.0 / n1), z, w)
    for prec, tol in ((zm.ZM_FP64, 1e-12), (zm.ZM_FP32_PAIRS, TOL32)):
        u = gpu_br(params(n1, n2, prec), z, w, gpu)
        err = relerr(u, ref)
        assert err < tol, (n1, n2, prec, err)
