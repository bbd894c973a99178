"""Cutoff BR solver over a seeded spread of meshes: sides 8..100, periods
1..3, periodic and free sheets, cutoffs from a few spacings up to the
largest a periodic cell allows.  Against the oracle (1e-12), and the
accepted-pair count against the definition's inclusion test written out
in numpy (exact: both sides take the same decisions bit for bit)."""
import numpy as np
import pytest

import oracle
import rocket_rig as rr
from zm_testutil import relerr, to_dev, to_host

pytestmark = pytest.mark.gpu


def cases(count=16, seed=77):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n1, n2 = (int(v) for v in rng.integers(8, 101, size=2))
        L1, L2 = (round(float(v), 3) for v in rng.uniform(1.0, 3.0, size=2))
        free = bool(i % 3 == 2)
        h = max(L1 / n1, L2 / n2)
        top = 0.45 * min(L1, L2) if not free else 0.6 * max(L1, L2)
        rc = round(float(rng.uniform(2.0 * h, top)), 4)
        out.append((i, n1, n2, L1, L2, free, rc))
    return out


def accepted_pairs(z, rc, L1, L2, free):
    n = z.shape[1]
    total = 0
    for i in range(n):
        r1 = z[0, i] - z[0]
        r2 = z[1, i] - z[1]
        if not free:
            r1 = r1 - np.rint(r1 / L1) * L1
            r2 = r2 - np.rint(r2 / L2) * L2
        r3 = z[2, i] - z[2]
        total += int(np.count_nonzero(r1 * r1 + r2 * r2 + r3 * r3 < rc * rc))
    return total


@pytest.mark.parametrize("i,n1,n2,L1,L2,free,rc", cases())
def test_cutoff_shape_spread(gpu, i, n1, n2, L1, L2, free, rc):
    import paper_2406_05490_amd as zm
    import torch
    z, w = rr.random_state(n1, n2, seed=300 + i, height=0.1)
    z[0] *= L1 / 2.0
    z[1] *= L2 / 2.0
    if not free:
        z[0] += 0.31 * L1       # drift across the seam: wrapped cells and wrap counts
        z[1] -= 0.17 * L2
    eps = 0.5 * min(L1 / n1, L2 / n2)
    bnd = zm.ZM_BOUNDARY_FREE if free else zm.ZM_BOUNDARY_PERIODIC
    p = zm.Params(n1, n2, eps=eps, period1=L1, period2=L2, cutoff=rc, boundary=bnd)
    ctx = zm.Context(p)
    ctx.profile_enable(True)
    ud = torch.empty(3 * p.n, dtype=torch.float64, device=gpu)
    ctx.br_velocity(to_dev(z, gpu), to_dev(w, gpu), ud)
    torch.cuda.synchronize()
    ref = oracle.br_velocity(oracle.Problem(n1, n2, eps=eps, period1=L1, period2=L2, cutoff=rc,
                                            boundary=1 if free else 0), z, w)
    assert relerr(to_host(ud, (3, p.n)), ref) < 1e-12
    assert ctx.cutoff_info().pairs_accepted == accepted_pairs(z, rc, L1, L2, free)
