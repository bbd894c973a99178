"""Limits of the GPU path (libzm.so through its C ABI) against the oracle:
the largest sides the library accepts (8192 for the BR paths, 4096 for the
FFT paths) on thin meshes, and the zero-step call.

Bar: 1e-12 normwise relative error for float64, 1e-5 for the FP32 pair form.
Sampled targets include the first and last points of the mesh and of the
long axis.
"""
import math

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


def oparams(p, **kw):
    return oracle.Problem(p.n1, p.n2, eps=p.eps, atwood=p.atwood, gravity=p.gravity, dt=p.dt,
                          nu=p.nu, period1=p.period1, period2=p.period2, cutoff=p.cutoff,
                          boundary=p.boundary, **kw)


def edge_targets(n1, n2, seed):
    N = n1 * n2
    idx = rr.sample_targets(N, 192, seed=seed)
    edges = [0, 1, n1 - 1, n1, N - n1, N - 1, N // 2, n1 * (n2 // 2) + n1 // 2]
    return np.unique(np.concatenate([idx, [e for e in edges if 0 <= e < N]]))


@pytest.mark.parametrize("n1,n2,kind", [
    (8192, 8, "exact"), (8, 8192, "exact"), (1024, 256, "fp32"), (8192, 64, "exact"),
    (8192, 8, "cutoff"), (8, 8192, "free"), (8192, 8, "free-cutoff"),
])
def test_largest_side_sampled(gpu, n1, n2, kind):
    import paper_2406_05490_amd as zm
    kw = dict(eps=0.5 * 2.0 / max(n1, n2) * 8)
    if kind == "fp32":
        kw["precision"] = zm.ZM_FP32_PAIRS
    if kind in ("cutoff", "free-cutoff"):
        kw["cutoff"] = 0.3
    if kind in ("free", "free-cutoff"):
        kw["boundary"] = zm.ZM_BOUNDARY_FREE
    p = zm.Params(n1, n2, **kw)
    z, w = rr.random_state(n1, n2, seed=n1 + 3 * n2, height=0.1)
    u = gpu_u(p, z, w, gpu)
    idx = edge_targets(n1, n2, seed=n2)
    ref = oracle.br_velocity(oparams(p), z, w, targets=idx)
    tol = 1e-5 if kind == "fp32" else TOL64
    assert relerr(u[:, idx], ref) < tol


def test_fp32_refused_where_its_bound_fails(gpu):
    """On 8192 x 8 the FP32 pair form would miss its bound (about 2e-4
    measured before the rule); the context is refused, FP64 serves."""
    import paper_2406_05490_amd as zm
    with pytest.raises(zm.ZMError) as e:
        zm.Context(zm.Params(8192, 8, eps=1e-3, precision=zm.ZM_FP32_PAIRS))
    assert e.value.status == zm.ZM_ERR_UNSUPPORTED


@pytest.mark.parametrize("n1,n2", [(4096, 8), (8, 4096), (4096, 16)])
def test_low_order_largest_side(gpu, n1, n2):
    import paper_2406_05490_amd as zm
    p = zm.Params(n1, n2, eps=1.0 / 64, model=zm.ZM_MODEL_LOW)
    z, w = rr.random_state(n1, n2, seed=n1 + n2, height=0.1)
    assert relerr(gpu_u(p, z, w, gpu), fft_reference(n1, n2, z, w)) < TOL64


@pytest.mark.parametrize("model", ["high", "low", "cutoff"])
def test_zero_steps_leave_state_bitwise(gpu, model):
    import paper_2406_05490_amd as zm
    import torch
    n = 32
    kw = {"low": dict(model=zm.ZM_MODEL_LOW), "cutoff": dict(cutoff=0.3), "high": {}}[model]
    p = zm.Params(n, n, eps=1.0 / n, **kw)
    z, w = rr.random_state(n, n, seed=4, height=0.1)
    ctx = zm.Context(p)
    ctx.init_state(to_dev(z, gpu), to_dev(w, gpu))
    ctx.step(0)
    z1 = torch.empty(3 * p.n, dtype=torch.float64, device=gpu)
    w1 = torch.empty(2 * p.n, dtype=torch.float64, device=gpu)
    ctx.get_state(z1, w1)
    torch.cuda.synchronize()
    assert np.array_equal(to_host(z1, (3, p.n)), z) and np.array_equal(to_host(w1, (2, p.n)), w)


def test_negative_steps_rejected(gpu):
    import paper_2406_05490_amd as zm
    p = zm.Params(16, 16, eps=1.0 / 16)
    ctx = zm.Context(p)
    with pytest.raises(zm.ZMError) as e:
        ctx.step(-1)
    assert e.value.status == zm.ZM_ERR_INVALID_ARG
