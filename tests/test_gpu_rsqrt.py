"""The FP64 pair kernels form (|r|^2 + eps^2)^(-3/2) from the hardware
reciprocal square root and one correction step, whose truncation leaves a
relative bias of about 15 e^2 / 8 <= 2.7e-14 per pair (e the hardware
estimate's error).  These tests exercise that step over squared distances
spanning many binades -- periods from 1e-3 to 1e3 and desingularisation
lengths from 0.02 to 8 mesh spacings -- and hold the FP64 BR velocity to the
oracle's (which takes 1 / sqrt(s) in plain FP64) at 1e-12, and the FP32 pair
form at 1e-5."""
import numpy as np
import pytest

import rocket_rig as rr
from zm_testutil import relerr, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("period", [1e-3, 1.0, 1e3])
@pytest.mark.parametrize("eps_over_h", [0.02, 0.5, 8.0])
def test_br_over_binades_matches_oracle(gpu, period, eps_over_h):
    import oracle
    import paper_2406_05490_amd as zm
    import torch
    n1, n2 = 40, 34
    z, w = rr.random_state(n1, n2, seed=77, height=0.08)
    z = z * (period / 2.0)              # positions on a period-`period` cell
    h = period / n1
    for prec, tol in ((zm.ZM_FP64, 1e-12), (zm.ZM_FP32_PAIRS, 1e-5)):
        p = zm.Params(n1, n2, eps=eps_over_h * h, period1=period, period2=period, precision=prec)
        ctx = zm.Context(p)
        zd, wd = to_dev(z, gpu), to_dev(w, gpu)
        u = torch.empty_like(zd)
        ctx.br_velocity(zd, wd, u)
        torch.cuda.synchronize()
        P = oracle.Problem(n1, n2, eps=p.eps, period1=period, period2=period)
        ref = oracle.br_velocity(P, z, w)
        err = relerr(to_host(u).reshape(3, -1), ref)
        assert err < tol, (period, eps_over_h, prec, err)
        assert np.all(np.isfinite(to_host(u)))
