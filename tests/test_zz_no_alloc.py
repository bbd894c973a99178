"""The allocation-free BR evaluation (zm_br_velocity_noalloc, scratch in the
library's static device array) against the context entry point
zm_br_velocity on the same inputs: several calls in a row on one device, each
later one on a smaller mesh than the one before, so that every call finds the
array holding the previous call's larger scratch.  FP64 within 1e-12 and the
FP32 pair form within 1e-5 (normwise relative); bitwise wherever the context's
launch shape fits the array (the same kernels then sum in the same order)."""
import numpy as np
import pytest

import rocket_rig as rr
from zm_testutil import relerr, to_dev, to_host

pytestmark = pytest.mark.gpu


def context_velocity(zm, p, zd, wd):
    import torch
    ctx = zm.Context(p)
    u = torch.empty_like(zd)
    ctx.br_velocity(zd, wd, u)
    torch.cuda.synchronize()
    out = to_host(u)
    del ctx
    return out, ctx_fits(zm, p)


def ctx_fits(zm, p):
    """True when the context's partial sums fit the static array, i.e. the
    allocation-free call takes the context's own launch shape."""
    R, S = zm.tuning_get(p.n1, p.n2, p.precision)
    N = p.n
    ties = p.boundary == zm.ZM_BOUNDARY_PERIODIC and (p.n1 % 2 == 0 or p.n2 % 2 == 0)

    def up(x):
        return (x + 255) // 256 * 256
    need = up(24 * N) + up(8 * N) + (up(48 * N) if ties else 0) + up(S * 24 * N)
    return need <= zm.NOALLOC_SCRATCH_BYTES


CASES = [
    # (n1, n2, precision, boundary, image_layers): each smaller than the one before
    (256, 256, "fp64", "periodic", 0),     # partial sums exceed the array: fewer source ranges
    (160, 150, "fp32", "periodic", 0),
    (96, 80, "fp64", "periodic", 1),
    (64, 64, "fp32", "free", 0),
    (45, 37, "fp64", "periodic", 0),       # odd sides: no tie corrections
    (24, 20, "fp32", "periodic", 0),
]


@pytest.mark.parametrize("order", ["descending", "repeat"])
def test_noalloc_matches_context_on_shrinking_meshes(gpu, order):
    import paper_2406_05490_amd as zm
    import torch
    cases = CASES if order == "descending" else [CASES[0], CASES[4], CASES[0], CASES[5]]
    for k, (n1, n2, prec, boundary, K) in enumerate(cases):
        precision = zm.ZM_FP64 if prec == "fp64" else zm.ZM_FP32_PAIRS
        bnd = zm.ZM_BOUNDARY_PERIODIC if boundary == "periodic" else zm.ZM_BOUNDARY_FREE
        p = zm.Params(n1, n2, eps=1.0 / n1, precision=precision, boundary=bnd, image_layers=K)
        z, w = rr.random_state(n1, n2, seed=40 + k, height=0.05)
        zd, wd = to_dev(z, gpu), to_dev(w, gpu)
        u = torch.full_like(zd, float("nan"))
        print(f"noalloc call {k}: {n1}x{n2} {prec} {boundary} K={K}", flush=True)
        zm.br_velocity_noalloc(p, zd, wd, u)
        torch.cuda.synchronize()
        got = to_host(u)
        ref, same_shape = context_velocity(zm, p, zd, wd)
        assert np.all(np.isfinite(got)), (n1, n2)
        tol = 1e-12 if prec == "fp64" else 1e-5
        assert relerr(got, ref) < tol, (n1, n2, prec, relerr(got, ref))
        if same_shape:
            assert np.array_equal(got, ref), (n1, n2, prec)


def test_noalloc_refuses_what_it_cannot_hold(gpu):
    import paper_2406_05490_amd as zm
    import torch
    n = 1024                                  # even sides: about 104 MiB of scratch
    p = zm.Params(n, n, eps=1.0 / n)
    zd = torch.zeros(3 * n * n, dtype=torch.float64, device=gpu)
    wd = torch.zeros(2 * n * n, dtype=torch.float64, device=gpu)
    u = torch.empty_like(zd)
    with pytest.raises(zm.ZMError) as e:
        zm.br_velocity_noalloc(p, zd, wd, u)
    assert e.value.status == zm.ZM_ERR_CAPACITY and "scratch" in str(e.value)
    with pytest.raises(zm.ZMError) as e:
        zm.br_velocity_noalloc(zm.Params(64, 64, eps=1 / 64, cutoff=0.2), zd[:3 * 4096],
                               wd[:2 * 4096], u[:3 * 4096])
    assert e.value.status == zm.ZM_ERR_UNSUPPORTED
