"""BR velocity against the oracle over a seeded spread of mesh shapes:
sides 8..130 (odd and even, so with and without tie lines), periods 1..3
(anisotropic spacings), with and without one extra image layer, in both
pair forms.  Patch, near-box, antipodal-band and whole-row-band cases all
occur somewhere in the spread.  Bars: 1e-12 (FP64), 1e-5 (FP32 pairs, on
the meshes where the library accepts that form)."""
import numpy as np
import pytest

import oracle
import rocket_rig as rr
from zm_testutil import relerr, to_dev, to_host

pytestmark = pytest.mark.gpu


def cases(count=24, seed=2026):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n1, n2 = (int(v) for v in rng.integers(8, 131, size=2))
        L1, L2 = (float(v) for v in rng.uniform(1.0, 3.0, size=2))
        K = int(rng.integers(0, 2)) if n1 * n2 <= 2500 else 0
        out.append((i, n1, n2, round(L1, 3), round(L2, 3), K))
    return out


def gpu_u(p, z, w, device):
    import paper_2406_05490_amd as zm
    import torch
    ctx = zm.Context(p)
    ud = torch.empty(3 * p.n, dtype=torch.float64, device=device)
    ctx.br_velocity(to_dev(z, device), to_dev(w, device), ud)
    torch.cuda.synchronize()
    return to_host(ud, (3, p.n))


@pytest.mark.parametrize("i,n1,n2,L1,L2,K", cases())
def test_br_velocity_shape_spread(gpu, i, n1, n2, L1, L2, K):
    import paper_2406_05490_amd as zm
    z, w = rr.random_state(n1, n2, seed=100 + i, height=0.1)
    z[0] *= L1 / 2.0
    z[1] *= L2 / 2.0
    eps = 0.5 * min(L1 / n1, L2 / n2)
    ref = oracle.br_velocity(oracle.Problem(n1, n2, eps=eps, images=K, period1=L1, period2=L2),
                             z, w)
    p64 = zm.Params(n1, n2, eps=eps, period1=L1, period2=L2, image_layers=K)
    assert relerr(gpu_u(p64, z, w, gpu), ref) < 1e-12
    p32 = zm.Params(n1, n2, eps=eps, period1=L1, period2=L2, image_layers=K,
                    precision=zm.ZM_FP32_PAIRS)
    if zm.workspace_bytes(p32) == 0:     # the FP32 form refused on this mesh
        return
    assert relerr(gpu_u(p32, z, w, gpu), ref) < 1e-5
