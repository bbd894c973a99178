"""Batched ensembles and graph replay: every instance of a batch matches its
solo run bitwise, and graph replays match eager steps bitwise."""
import numpy as np
import pytest

import oracle
import rocket_rig as rr
from zm_testutil import relerr, to_dev, to_host

pytestmark = pytest.mark.gpu


def member_params(m, precision):
    import paper_2406_05490_amd as zm
    return zm.Params(m.n, m.n, eps=m.eps, atwood=m.atwood, gravity=1.0, dt=1e-3,
                     precision=precision)


def solo_run(p, z, w, steps, device, flags=0):
    import paper_2406_05490_amd as zm
    import torch
    q = zm.Params(**{**p.__dict__, "flags": flags})
    ctx = zm.Context(q)
    zd, wd = to_dev(z, device), to_dev(w, device)
    ctx.init_state(zd, wd)
    ctx.step(steps)
    z1 = torch.empty_like(zd); w1 = torch.empty_like(wd)
    ctx.get_state(z1, w1)
    torch.cuda.synchronize()
    return to_host(z1, (3, -1)), to_host(w1, (2, -1))


def batch_states(b, ps, device):
    import torch
    out = []
    for i, p in enumerate(ps):
        z1 = torch.empty(3 * p.n, dtype=torch.float64, device=device)
        w1 = torch.empty(2 * p.n, dtype=torch.float64, device=device)
        b.get_state(i, z1, w1)
        out.append((z1, w1))
    torch.cuda.synchronize()
    return [(to_host(z, (3, -1)), to_host(w, (2, -1))) for z, w in out]


def mixed_members():
    import paper_2406_05490_amd as zm
    ms = [rr.Member(32, 0.3, 0.05), rr.Member(48, 0.7, 0.02), rr.Member(17, 0.5, 0.08),
          rr.Member(64, 0.2, 0.1), rr.Member(40, 0.9, 0.04)]
    precs = [zm.ZM_FP32_PAIRS, zm.ZM_FP64, zm.ZM_FP32_PAIRS, zm.ZM_FP64, zm.ZM_FP32_PAIRS]
    return ms, precs


@pytest.mark.parametrize("graph", [False, True])
def test_batch_matches_solo_bitwise(gpu, graph):
    import paper_2406_05490_amd as zm
    ms, precs = mixed_members()
    ps = [member_params(m, pr) for m, pr in zip(ms, precs)]
    b = zm.Batch(ps, flags=zm.ZM_FLAG_GRAPH if graph else 0)
    states = [m.state() for m in ms]
    for i, (z, w) in enumerate(states):
        b.init_state(i, to_dev(z, gpu), to_dev(w, gpu))
    b.step(3)
    got = batch_states(b, ps, gpu)
    for i, (p, (z, w)) in enumerate(zip(ps, states)):
        zs, ws = solo_run(p, z, w, 3, gpu)
        assert np.array_equal(got[i][0], zs) and np.array_equal(got[i][1], ws), f"instance {i}"


def test_batch_fp64_member_matches_oracle(gpu):
    import paper_2406_05490_amd as zm
    ms, precs = mixed_members()
    ps = [member_params(m, pr) for m, pr in zip(ms, precs)]
    b = zm.Batch(ps)
    states = [m.state() for m in ms]
    for i, (z, w) in enumerate(states):
        b.init_state(i, to_dev(z, gpu), to_dev(w, gpu))
    b.step(2)
    got = batch_states(b, ps, gpu)
    i = 1                                   # 48 x 48, FP64
    P = oracle.Problem(ps[i].n1, ps[i].n2, eps=ps[i].eps, atwood=ps[i].atwood, dt=ps[i].dt)
    zr, wr = oracle.rk3(P, *states[i], 2)
    assert relerr(got[i][0], zr) < 1e-12 and relerr(got[i][1], wr) < 1e-12
    j = 2                                   # 17 x 17, FP32 pairs: motion within 1e-5
    P = oracle.Problem(ps[j].n1, ps[j].n2, eps=ps[j].eps, atwood=ps[j].atwood, dt=ps[j].dt)
    zr, wr = oracle.rk3(P, *states[j], 2)
    assert relerr(got[j][0] - states[j][0], zr - states[j][0]) < 1e-5


def test_graph_replays_match_eager_each_step(gpu):
    """Replay a captured step several times, with eager work and
    synchronisations in between, and compare every replay with eager steps."""
    import paper_2406_05490_amd as zm
    import torch
    ms, precs = mixed_members()
    ps = [member_params(m, pr) for m, pr in zip(ms, precs)]
    eager = zm.Batch(ps)
    graph = zm.Batch(ps, flags=zm.ZM_FLAG_GRAPH)
    states = [m.state() for m in ms]
    for i, (z, w) in enumerate(states):
        eager.init_state(i, to_dev(z, gpu), to_dev(w, gpu))
        graph.init_state(i, to_dev(z, gpu), to_dev(w, gpu))
    for rep in range(4):
        graph.step(1)
        torch.cuda.synchronize()
        scratch = torch.randn(1 << 16, device=gpu).sum()   # unrelated eager work
        eager.step(1)
        a, b = batch_states(eager, ps, gpu), batch_states(graph, ps, gpu)
        for i in range(len(ps)):
            assert np.array_equal(a[i][0], b[i][0]) and np.array_equal(a[i][1], b[i][1]), \
                f"replay {rep} instance {i}"
        del scratch


def test_solo_graph_matches_eager(gpu):
    import paper_2406_05490_amd as zm
    for prec in (zm.ZM_FP64, zm.ZM_FP32_PAIRS):
        p = zm.Params(64, 48, eps=1 / 64, atwood=0.5, dt=1e-3, precision=prec)
        z, w = rr.single_mode(64, 48, 0.05, noise=1e-4, seed=1)
        a = solo_run(p, z, w, 3, gpu)
        b = solo_run(p, z, w, 3, gpu, flags=zm.ZM_FLAG_GRAPH)
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_ensemble64_sampled_members_match_solo(gpu):
    """The 64-member uneven ensemble (FP32 form, graph-captured): 2 steps,
    six sampled members compared bitwise with their solo runs."""
    import paper_2406_05490_amd as zm
    ms = rr.ensemble(64, seed=3)
    ps = [member_params(m, zm.ZM_FP32_PAIRS) for m in ms]
    b = zm.Batch(ps, flags=zm.ZM_FLAG_GRAPH)
    info = b.info()
    assert info.count == 64 and info.work_items[1] > 0 and info.work_items[0] == 0
    states = [m.state() for m in ms]
    for i, (z, w) in enumerate(states):
        b.init_state(i, to_dev(z, gpu), to_dev(w, gpu))
    b.step(2)
    got = batch_states(b, ps, gpu)
    for i in (0, 7, 19, 33, 50, 63):
        zs, ws = solo_run(ps[i], *states[i], 2, gpu)
        assert np.array_equal(got[i][0], zs) and np.array_equal(got[i][1], ws), f"member {i}"


def test_batch_argument_errors(gpu):
    import paper_2406_05490_amd as zm
    import torch
    ps = [zm.Params(16, 16, eps=1 / 16), zm.Params(24, 16, eps=1 / 24)]
    b = zm.Batch(ps)
    z = torch.zeros(3 * 256, dtype=torch.float64, device=gpu)
    w = torch.zeros(2 * 256, dtype=torch.float64, device=gpu)
    lib = zm.load()
    assert lib.zm_batch_init_state(b.handle, 2, z.data_ptr(), w.data_ptr()) == zm.ZM_ERR_INVALID_ARG
    assert lib.zm_batch_step(b.handle, -1) == zm.ZM_ERR_INVALID_ARG
    with pytest.raises(zm.ZMError):
        zm.Batch([zm.Params(16, 16, eps=1 / 16, flags=zm.ZM_FLAG_GRAPH)])
