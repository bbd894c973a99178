"""Launch-shape variants and the autotuner: every shape computes the same
velocities (to the parity bar), and tuned shapes apply to solo contexts and
batch members alike."""
import numpy as np
import pytest

import oracle
import rocket_rig as rr
from zm_testutil import relerr, to_dev, to_host

pytestmark = pytest.mark.gpu


def br(p, z, w, device):
    import paper_2406_05490_amd as zm
    import torch
    ctx = zm.Context(p)
    ud = torch.empty(3 * p.n, dtype=torch.float64, device=device)
    ctx.br_velocity(to_dev(z, device), to_dev(w, device), ud)
    torch.cuda.synchronize()
    info = ctx.launch_info()
    return to_host(ud, (3, -1)), (info.targets_per_lane, info.source_splits)


@pytest.mark.parametrize("prec_name,tol", [("ZM_FP64", 1e-12), ("ZM_FP32_PAIRS", 1e-5)])
@pytest.mark.parametrize("R,splits", [(1, 1), (1, 7), (2, 3), (2, 40), (4, 2), (4, 37)])
def test_every_shape_matches_oracle(gpu, prec_name, tol, R, splits):
    import paper_2406_05490_amd as zm
    prec = getattr(zm, prec_name)
    n1, n2 = 40, 37
    z, w = rr.random_state(n1, n2, seed=21, height=0.1)
    p = zm.Params(n1, n2, eps=1 / n1, precision=prec)
    ref = oracle.br_velocity(oracle.Problem(n1, n2, eps=p.eps), z, w)
    try:
        zm.tuning_set(n1, n2, prec, R, splits)
        u, shape = br(p, z, w, gpu)
        assert shape == (R, min(splits, n2))
        assert relerr(u, ref) < tol
    finally:
        zm.tuning_set(n1, n2, prec)


def test_autotune_then_solo_equals_batch(gpu):
    import paper_2406_05490_amd as zm
    import torch
    n = 96
    p = zm.Params(n, n, eps=1 / n, precision=zm.ZM_FP32_PAIRS, atwood=0.4)
    try:
        R, S, ms = zm.autotune(p)
        assert R in (1, 2, 4) and 1 <= S <= n and ms > 0
        assert zm.tuning_get(n, n, zm.ZM_FP32_PAIRS) == (R, S)
        z, w = rr.single_mode(n, n, 0.05)
        ctx = zm.Context(p)
        zd, wd = to_dev(z, gpu), to_dev(w, gpu)
        ctx.init_state(zd, wd)
        ctx.step(2)
        zs = torch.empty_like(zd); ws = torch.empty_like(wd)
        ctx.get_state(zs, ws)
        other = zm.Params(48, 48, eps=1 / 48, precision=zm.ZM_FP32_PAIRS)
        b = zm.Batch([other, p])
        z2, w2 = rr.single_mode(48, 48, 0.02)
        b.init_state(0, to_dev(z2, gpu), to_dev(w2, gpu))
        b.init_state(1, zd, wd)
        b.step(2)
        zb = torch.empty_like(zd); wb = torch.empty_like(wd)
        b.get_state(1, zb, wb)
        torch.cuda.synchronize()
        assert torch.equal(zs, zb) and torch.equal(ws, wb)
    finally:
        zm.tuning_set(n, n, zm.ZM_FP32_PAIRS)
