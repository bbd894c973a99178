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


def test_batch_autotune_sets_shapes_the_batch_and_solo_runs_share(gpu):
    """The batch tuner times the batched sweep itself and stores one shape per
    mesh size; members of one size share it, the table holds it, and a batch
    built afterwards equals solo contexts bitwise and the oracle at the
    parity bar."""
    import paper_2406_05490_amd as zm
    import torch
    sizes = [(32, zm.ZM_FP32_PAIRS), (48, zm.ZM_FP64), (32, zm.ZM_FP32_PAIRS), (64, zm.ZM_FP32_PAIRS),
             (40, zm.ZM_FP64)]
    ps = [zm.Params(n, n, eps=1 / n, precision=pr, atwood=0.3 + 0.1 * i)
          for i, (n, pr) in enumerate(sizes)]
    keys = {(p.n1, p.n2, p.precision) for p in ps}
    try:
        shapes, ms = zm.batch_autotune(ps)
        assert ms > 0 and len(shapes) == len(ps)
        for p, (R, S) in zip(ps, shapes):
            assert R in (1, 2, 4) and 1 <= S <= p.n2
            assert zm.tuning_get(p.n1, p.n2, p.precision) == (R, S)
        assert shapes[0] == shapes[2]                 # one shape per size
        b = zm.Batch(ps)
        states = []
        for i, p in enumerate(ps):
            z, w = rr.random_state(p.n1, p.n2, seed=60 + i, height=0.05)
            states.append((z, w))
            b.init_state(i, to_dev(z, gpu), to_dev(w, gpu))
        b.step(2)
        for i, p in enumerate(ps):
            z, w = states[i]
            zb = torch.empty(3 * p.n, dtype=torch.float64, device=gpu)
            wb = torch.empty(2 * p.n, dtype=torch.float64, device=gpu)
            b.get_state(i, zb, wb)
            ctx = zm.Context(p)
            ctx.init_state(to_dev(z, gpu), to_dev(w, gpu))
            ctx.step(2)
            zs, ws = torch.empty_like(zb), torch.empty_like(wb)
            ctx.get_state(zs, ws)
            torch.cuda.synchronize()
            assert torch.equal(zs, zb) and torch.equal(ws, wb), i
            assert ctx.launch_info().source_splits == shapes[i][1]
            P = oracle.Problem(p.n1, p.n2, eps=p.eps, atwood=p.atwood, gravity=p.gravity, dt=p.dt)
            zr, wr = oracle.rk3(P, z, w, 2)
            tol = 1e-9 if p.precision == zm.ZM_FP64 else 1e-5
            assert relerr(to_host(zb).reshape(3, -1) - z, zr - z) < tol, i
    finally:
        for (n1, n2, pr) in keys:
            zm.tuning_set(n1, n2, pr)
