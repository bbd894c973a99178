"""The right-hand side (z_t, w_t) of the low-order, medium-order and
free-sheet models against the oracle over a seeded spread of meshes: sides
(powers of two for the FFT models, any for the free sheet), periods 1..3,
Atwood numbers, gravity and viscosity.  Bar: 1e-12 normwise (FP64)."""
import numpy as np
import pytest

import oracle
import rocket_rig as rr
from zm_testutil import relerr, to_dev, to_host

pytestmark = pytest.mark.gpu


def cases(kind, count, seed):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        if kind == "free":
            n1, n2 = (int(v) for v in rng.integers(8, 97, size=2))
        else:
            n1, n2 = (int(2 ** v) for v in rng.integers(3, 8, size=2))
        L1, L2 = (round(float(v), 3) for v in rng.uniform(1.0, 3.0, size=2))
        A = round(float(rng.uniform(-0.9, 0.9)), 3)
        g = round(float(rng.uniform(0.5, 2.0)), 3)
        nu = 0.0 if i % 2 == 0 else 1e-3
        out.append((kind, i, n1, n2, L1, L2, A, g, nu))
    return out


ALL = cases("low", 10, 501) + cases("medium", 6, 502) + cases("free", 8, 503)


@pytest.mark.parametrize("kind,i,n1,n2,L1,L2,A,g,nu", ALL)
def test_rhs_model_spread(gpu, kind, i, n1, n2, L1, L2, A, g, nu):
    import paper_2406_05490_amd as zm
    import torch
    z, w = rr.random_state(n1, n2, seed=700 + i, height=0.1)
    z[0] *= L1 / 2.0
    z[1] *= L2 / 2.0
    eps = 0.5 * min(L1 / n1, L2 / n2)
    model = {"low": zm.ZM_MODEL_LOW, "medium": zm.ZM_MODEL_MEDIUM, "free": zm.ZM_MODEL_HIGH}[kind]
    free = kind == "free"
    p = zm.Params(n1, n2, eps=eps, period1=L1, period2=L2, atwood=A, gravity=g, nu=nu,
                  model=model, boundary=zm.ZM_BOUNDARY_FREE if free else zm.ZM_BOUNDARY_PERIODIC)
    ctx = zm.Context(p)
    zd, wd = to_dev(z, gpu), to_dev(w, gpu)
    zt = torch.empty_like(zd); wt = torch.empty_like(wd)
    ctx.rhs(zd, wd, zt, wt)
    torch.cuda.synchronize()
    P = oracle.Problem(n1, n2, eps=eps, atwood=A, gravity=g, nu=nu, period1=L1, period2=L2,
                       model=int(model), boundary=1 if free else 0)
    rz, rw = oracle.rhs(P, z, w)
    assert relerr(to_host(zt, (3, -1)), rz) < 1e-12
    assert relerr(to_host(wt, (2, -1)), rw) < 1e-12
