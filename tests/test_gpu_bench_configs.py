"""Parity at the sizes and in the configurations the benchmark times for the
cutoff, free-sheet, low- and medium-order paths (libzm.so through its C
ABI), on sampled targets the oracle evaluates one by one, or against numpy's
FFT of the definition where the oracle's direct DFT would take hours.

Bar: 1e-12 normwise relative error (float64 throughout).
"""
import numpy as np
import pytest

import oracle
import rocket_rig as rr
from zm_testutil import fft_reference, relerr, to_dev, to_host

pytestmark = pytest.mark.gpu

TOL64 = 1e-12


def gpu_u(p, z, w, device):
    import paper_2406_05490_amd as zm
    import torch
    ctx = zm.Context(p)
    ud = torch.empty(3 * p.n, dtype=torch.float64, device=device)
    ctx.br_velocity(to_dev(z, device), to_dev(w, device), ud)
    torch.cuda.synchronize()
    return to_host(ud, (3, p.n))


def gpu_rhs(p, z, w, device):
    import paper_2406_05490_amd as zm
    import torch
    ctx = zm.Context(p)
    zt = torch.empty(3 * p.n, dtype=torch.float64, device=device)
    wt = torch.empty(2 * p.n, dtype=torch.float64, device=device)
    ctx.rhs(to_dev(z, device), to_dev(w, device), zt, wt)
    torch.cuda.synchronize()
    return to_host(zt, (3, p.n)), to_host(wt, (2, p.n))


def oparams(p):
    return oracle.Problem(p.n1, p.n2, eps=p.eps, atwood=p.atwood, gravity=p.gravity, dt=p.dt,
                          nu=p.nu, period1=p.period1, period2=p.period2, cutoff=p.cutoff,
                          boundary=p.boundary)


def sampled(n, seed):
    idx = rr.sample_targets(n * n, 256, seed=seed)
    return np.unique(np.concatenate([idx, [0, n - 1, n * n - n, n * n - 1]]))


@pytest.mark.parametrize("name,n,rc,free", [
    ("multimode768", 768, 0.2 * 2.0 / 6.0, False),
    ("singlemode512", 512, 0.5 * 2.0 / 6.0, False),
    ("free_singlemode512", 512, 1.0 / 6.0, True),
])
def test_cutoff_bench_configs_sampled(gpu, name, n, rc, free):
    import paper_2406_05490_amd as zm
    if name.startswith("multimode"):
        z, _ = rr.multi_mode(n, n, 8, seed=1)
        w = rr.synthetic_vorticity(n, n, seed=1)
    else:
        z, _ = rr.single_mode(n, n, 0.05)
        w = rr.synthetic_vorticity(n, n, seed=2)
    p = zm.Params(n, n, eps=1.0 / n, cutoff=rc,
                  boundary=zm.ZM_BOUNDARY_FREE if free else zm.ZM_BOUNDARY_PERIODIC)
    u = gpu_u(p, z, w, gpu)
    idx = sampled(n, seed=n)
    assert relerr(u[:, idx], oracle.br_velocity(oparams(p), z, w, targets=idx)) < TOL64


def test_low_order_4096_against_numpy_fft(gpu):
    """The low-order benchmark configuration (4096 x 4096, eight modes)."""
    import paper_2406_05490_amd as zm
    n = 4096
    z, _ = rr.multi_mode(n, n, 8, seed=1)
    w = rr.synthetic_vorticity(n, n, seed=1)
    p = zm.Params(n, n, eps=1.0 / n, model=zm.ZM_MODEL_LOW)
    assert relerr(gpu_u(p, z, w, gpu), fft_reference(n, n, z, w)) < TOL64


@pytest.mark.parametrize("n,rc", [(512, 0.0), (1024, 0.2 * 2.0 / 6.0)])
def test_medium_bench_configs(gpu, n, rc):
    """Medium order at the benchmark sizes: the sheet velocity (= the BR
    velocity) against the oracle on sampled targets; the vorticity derivative
    against the oracle's V and difference stencil fed numpy's FFT velocity
    (the oracle's direct DFT would take hours here), and bit for bit equal to
    the low-order model's on the same state (both take V from the same FFT
    velocity)."""
    import paper_2406_05490_amd as zm
    z, _ = rr.multi_mode(n, n, 8, seed=1)
    w = rr.synthetic_vorticity(n, n, seed=1)
    pm = zm.Params(n, n, eps=1.0 / n, cutoff=rc, model=zm.ZM_MODEL_MEDIUM)
    zt, wt = gpu_rhs(pm, z, w, gpu)
    idx = sampled(n, seed=n + 1)
    ref = oracle.br_velocity(oparams(pm), z, w, targets=idx)
    assert relerr(zt[:, idx], ref) < TOL64
    wref = oracle.wt_sampled(oparams(pm), z, w, fft_reference(n, n, z, w), idx)
    assert relerr(wt[:, idx], wref) < TOL64
    _, wt_low = gpu_rhs(zm.Params(n, n, eps=1.0 / n, model=zm.ZM_MODEL_LOW), z, w, gpu)
    assert np.array_equal(wt, wt_low)
