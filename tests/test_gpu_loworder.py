"""Low-order model on the GPU (libzm.so through its C ABI) against the oracle.

Bar: 1e-12 normwise relative error in float64 on the same seeded inputs.
The oracle evaluates the Riesz transforms by direct DFT sums (O(N^2)), so
the full-field comparisons stop at 64 x 64; at 1024 x 1024 the GPU result is
compared with numpy's FFT of the same definition (that reference is checked
against the oracle at small sizes in the oracle's own pins).
"""
import math

import numpy as np
import pytest

import oracle
import rocket_rig as rr
from zm_testutil import fft_reference, relerr, to_dev, to_host

pytestmark = pytest.mark.gpu

TOL64 = 1e-12


def params(n1, n2, **kw):
    import paper_2406_05490_amd as zm
    kw.setdefault("eps", 0.5 * 2.0 / n1)
    return zm.Params(n1, n2, model=zm.ZM_MODEL_LOW, **kw)


def oparams(p):
    return oracle.Problem(p.n1, p.n2, eps=p.eps, atwood=p.atwood, gravity=p.gravity, dt=p.dt,
                          nu=p.nu, period1=p.period1, period2=p.period2, model=1)


def gpu_u(p, z, w, device):
    import paper_2406_05490_amd as zm
    import torch
    ctx = zm.Context(p)
    ud = torch.empty(3 * p.n, dtype=torch.float64, device=device)
    ctx.br_velocity(to_dev(z, device), to_dev(w, device), ud)
    torch.cuda.synchronize()
    return to_host(ud, (3, p.n))


@pytest.mark.parametrize("n1,n2,L1,L2,seed", [
    (16, 16, 2.0, 2.0, 0), (32, 8, 2.0, 2.0, 1), (64, 64, 2.0, 2.0, 2), (8, 64, 2.0, 2.0, 3),
    (32, 16, 3.0, 1.5, 4),
])
def test_low_order_velocity_matches_oracle(gpu, n1, n2, L1, L2, seed):
    p = params(n1, n2, period1=L1, period2=L2)
    z, w = rr.random_state(n1, n2, seed=seed, height=0.1)
    z[0] *= L1 / 2.0
    z[1] *= L2 / 2.0
    assert relerr(gpu_u(p, z, w, gpu), oracle.br_velocity(oparams(p), z, w)) < TOL64


def test_low_order_flat_sheet_symbol(gpu):
    n = 64
    p = params(n, n)
    z, _ = rr.flat_state(n, n)
    A1, A2 = rr.grid(n, n)
    k1, k2 = 3 * math.pi, -2 * math.pi
    mu = np.cos(k1 * A1 + k2 * A2).ravel()
    s = np.sin(k1 * A1 + k2 * A2).ravel()
    u = gpu_u(p, z, np.stack([-k1 * s, -k2 * s]), gpu)
    assert np.max(np.abs(u[:2])) == 0.0
    assert np.max(np.abs(u[2] + 0.5 * math.hypot(k1, k2) * mu)) < 1e-12 * math.hypot(k1, k2)


def test_low_order_rhs_matches_oracle(gpu):
    import paper_2406_05490_amd as zm
    import torch
    n1, n2 = 32, 16
    p = params(n1, n2, atwood=0.7, gravity=1.3, nu=1e-3)
    z, w = rr.random_state(n1, n2, seed=5, height=0.1)
    ctx = zm.Context(p)
    zt = torch.empty(3 * p.n, dtype=torch.float64, device=gpu)
    wt = torch.empty(2 * p.n, dtype=torch.float64, device=gpu)
    ctx.rhs(to_dev(z, gpu), to_dev(w, gpu), zt, wt)
    torch.cuda.synchronize()
    ozt, owt = oracle.rhs(oparams(p), z, w)
    assert relerr(to_host(zt, (3, p.n)), ozt) < TOL64
    assert relerr(to_host(wt, (2, p.n)), owt) < TOL64


@pytest.mark.parametrize("graph", [False, True])
def test_low_order_steps_match_oracle(gpu, graph):
    import paper_2406_05490_amd as zm
    import torch
    n = 32
    p = params(n, n, dt=5e-3, flags=zm.ZM_FLAG_GRAPH if graph else 0)
    z, _ = rr.multi_mode(n, n, 4, seed=6, noise=0.0)
    w = rr.synthetic_vorticity(n, n, seed=6, sigma=0.02)   # O(0.1) velocities from the start
    ctx = zm.Context(p)
    ctx.init_state(to_dev(z, gpu), to_dev(w, gpu))
    ctx.step(4)
    z1 = torch.empty(3 * p.n, dtype=torch.float64, device=gpu)
    w1 = torch.empty(2 * p.n, dtype=torch.float64, device=gpu)
    ctx.get_state(z1, w1)
    torch.cuda.synchronize()
    oz, ow = oracle.rk3(oparams(p), z, w, 4)
    assert relerr(to_host(z1, (3, p.n)) - z, oz - z) < 1e-11
    assert relerr(to_host(w1, (2, p.n)), ow) < 1e-11


def test_low_order_repeat_bitwise(gpu):
    n = 128
    p = params(n, n)
    z, w = rr.random_state(n, n, seed=7, height=0.05)
    assert np.array_equal(gpu_u(p, z, w, gpu), gpu_u(p, z, w, gpu))


def test_low_order_1024_against_numpy_fft(gpu):
    n = 1024
    p = params(n, n)
    z, _ = rr.multi_mode(n, n, 16, seed=2)
    w = rr.synthetic_vorticity(n, n, seed=2)
    u = gpu_u(p, z, w, gpu)
    W1 = np.fft.fft2(w[0].reshape(n, n))
    W2 = np.fft.fft2(w[1].reshape(n, n))
    m = np.fft.fftfreq(n, 1.0 / n)
    M1, M2 = np.meshgrid(m, m)
    K1, K2 = np.pi * M1, np.pi * M2
    KK = np.hypot(K1, K2)
    with np.errstate(invalid="ignore", divide="ignore"):
        c1 = np.where(KK > 0, K1 / KK, 0.0)
        c2 = np.where(KK > 0, K2 / KK, 0.0)
    c1[:, n // 2] = 0.0
    c2[n // 2, :] = 0.0
    S = np.real(np.fft.ifft2(0.5j * (c1 * W1 + c2 * W2))).ravel()
    t1, t2 = oracle.tangents(oracle.Problem(n, n, eps=1.0 / n), z)
    nrm = np.cross(t1.T, t2.T).T
    ref = S * (nrm / np.linalg.norm(nrm, axis=0))
    assert relerr(u, ref) < TOL64


@pytest.mark.parametrize("n1,n2,L1,L2", [(64, 4096, 0.5, 2.0), (4096, 64, 2.0, 0.5)])
def test_low_order_4096_side_against_numpy_fft(gpu, n1, n2, L1, L2):
    """A side of 4096: the symbol rows of a 4096-point column transform keep
    the row in registers between the forward FFT, the symbol and the inverse
    FFT (64 x 4096); the pack and inverse rows take 4096-point row transforms
    in LDS (4096 x 64).  Both against numpy's FFT of the definition."""
    p = params(n1, n2, period1=L1, period2=L2)
    z, _ = rr.multi_mode(n1, n2, 8, seed=5)
    z[0] *= L1 / 2.0
    z[1] *= L2 / 2.0
    w = rr.synthetic_vorticity(n1, n2, seed=5)
    u = gpu_u(p, z, w, gpu)
    assert relerr(u, fft_reference(n1, n2, z, w, L1, L2)) < TOL64
