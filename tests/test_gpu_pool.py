"""Serving pool: continuous batching with admission by footprint.  Each
request's trajectory is bitwise identical alone (a solo context) and in the
mix, whatever else is admitted, finishes, fails or is cancelled around it."""
import numpy as np
import pytest

import rocket_rig as rr
from zm_testutil import to_dev, to_host

pytestmark = pytest.mark.gpu


def req_params(n, atwood, precision):
    import paper_2406_05490_amd as zm
    return zm.Params(n, n, eps=1.0 / n, atwood=atwood, gravity=1.0, dt=1e-3, precision=precision)


def solo(p, z, w, steps, device):
    import paper_2406_05490_amd as zm
    import torch
    ctx = zm.Context(p)
    zd, wd = to_dev(z, device), to_dev(w, device)
    ctx.init_state(zd, wd)
    ctx.step(steps)
    z1 = torch.empty_like(zd); w1 = torch.empty_like(wd)
    ctx.get_state(z1, w1)
    torch.cuda.synchronize()
    return to_host(z1), to_host(w1)


def fetch(pool, rid, p, device):
    import torch
    z1 = torch.empty(3 * p.n, dtype=torch.float64, device=device)
    w1 = torch.empty(2 * p.n, dtype=torch.float64, device=device)
    pool.fetch(rid, z1, w1)
    torch.cuda.synchronize()
    return to_host(z1), to_host(w1)


def specs():
    import paper_2406_05490_amd as zm
    return [(48, 0.3, zm.ZM_FP32_PAIRS, 5, 0.05), (64, 0.7, zm.ZM_FP64, 3, 0.02),
            (40, 0.5, zm.ZM_FP32_PAIRS, 7, 0.08), (72, 0.2, zm.ZM_FP64, 4, 0.04),
            (32, 0.9, zm.ZM_FP32_PAIRS, 6, 0.03)]


def test_pool_same_alone_and_in_the_mix(gpu):
    """Budget for about two requests at a time: requests queue, are admitted
    as others finish, and overlap on the device; every result equals its
    solo run bitwise."""
    import paper_2406_05490_amd as zm
    reqs = []
    for n, a, prec, steps, amp in specs():
        p = req_params(n, a, prec)
        z, w = rr.single_mode(n, n, amp)
        reqs.append((p, z, w, steps))
    sizes = sorted(zm.pool_request_bytes(p) for p, *_ in reqs)
    pool = zm.Pool(sizes[-1] + sizes[-2])
    ids = [pool.submit(p, to_dev(z, gpu), to_dev(w, gpu), steps) for p, z, w, steps in reqs]
    index = {rid: i for i, rid in enumerate(ids)}
    results, seen_live = {}, []
    for _ in range(100):
        recs = pool.iterate()
        if not recs and pool.stats().queued == 0:
            break
        seen_live.append(len(recs))
        st = pool.stats()
        assert st.used_bytes <= st.budget_bytes
        for rid, done, state, ms in recs:
            assert ms > 0
            if state == zm.ZM_REQ_FINISHED:         # serve the result, return the budget
                assert done == reqs[index[rid]][3]
                results[rid] = fetch(pool, rid, reqs[index[rid]][0], gpu)
                pool.release(rid)
    assert max(seen_live) >= 2                     # requests overlapped on the device
    assert max(seen_live) < len(reqs)              # and the budget made some wait
    assert sorted(results) == sorted(ids)
    for rid, (p, z, w, steps) in zip(ids, reqs):
        ref = solo(p, z, w, steps, gpu)
        got = results[rid]
        assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1]), f"request {rid}"
    assert pool.stats().used_bytes == 0


def test_pool_admission_is_fifo_by_footprint(gpu):
    import paper_2406_05490_amd as zm
    big = req_params(96, 0.5, zm.ZM_FP64)
    small = req_params(32, 0.5, zm.ZM_FP64)
    zb, wb = rr.single_mode(96, 96, 0.05)
    zs, ws = rr.single_mode(32, 32, 0.05)
    pool = zm.Pool(zm.pool_request_bytes(big) + zm.pool_request_bytes(small))
    a = pool.submit(big, to_dev(zb, gpu), to_dev(wb, gpu), 3)
    b = pool.submit(big, to_dev(zb, gpu), to_dev(wb, gpu), 2)
    c = pool.submit(small, to_dev(zs, gpu), to_dev(ws, gpu), 2)
    recs = pool.iterate()
    # b does not fit next to a, and c may not overtake b (first in, first out)
    assert [r[0] for r in recs] == [a]
    assert pool.query(b)[0] == zm.ZM_REQ_QUEUED and pool.query(c)[0] == zm.ZM_REQ_QUEUED
    pool.iterate(); pool.iterate()                 # a finishes after its 3rd step
    assert pool.query(a) == (zm.ZM_REQ_FINISHED, 3)
    pool.release(a)
    recs = pool.iterate()                          # b and c fit together now
    assert sorted(r[0] for r in recs) == [b, c]


def test_pool_cancel_and_capacity(gpu):
    import paper_2406_05490_amd as zm
    p = req_params(48, 0.4, zm.ZM_FP32_PAIRS)
    z, w = rr.single_mode(48, 48, 0.05)
    q = req_params(40, 0.6, zm.ZM_FP64)
    zq, wq = rr.single_mode(40, 40, 0.03)
    pool = zm.Pool(zm.pool_request_bytes(p) + zm.pool_request_bytes(q))
    a = pool.submit(p, to_dev(z, gpu), to_dev(w, gpu), 4)
    b = pool.submit(q, to_dev(zq, gpu), to_dev(wq, gpu), 4)
    c = pool.submit(q, to_dev(zq, gpu), to_dev(wq, gpu), 4)   # queued: no room
    pool.iterate()
    pool.cancel(b)                                 # live
    pool.cancel(c)                                 # still queued, or admitted now
    assert pool.query(b)[0] == zm.ZM_REQ_UNKNOWN and pool.query(c)[0] == zm.ZM_REQ_UNKNOWN
    for _ in range(3):
        pool.iterate()
    assert pool.query(a) == (zm.ZM_REQ_FINISHED, 4)
    got = fetch(pool, a, p, gpu)
    ref = solo(p, z, w, 4, gpu)
    assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1])
    huge = req_params(512, 0.5, zm.ZM_FP64)
    zh, wh = rr.flat_state(512, 512)
    with pytest.raises(zm.ZMError) as e:
        pool.submit(huge, to_dev(zh, gpu), to_dev(wh, gpu), 1)
    assert e.value.status == zm.ZM_ERR_CAPACITY


def test_pool_evicts_failing_request_alone(gpu):
    import paper_2406_05490_amd as zm
    good = req_params(48, 0.5, zm.ZM_FP32_PAIRS)
    zg, wg = rr.single_mode(48, 48, 0.05)
    bad = req_params(32, 0.5, zm.ZM_FP64)
    zb, wb = rr.single_mode(32, 32, 0.05)
    zb[2, 100] = np.nan
    pool = zm.Pool(1 << 28, flags=zm.ZM_FLAG_CHECK_FINITE)
    a = pool.submit(good, to_dev(zg, gpu), to_dev(wg, gpu), 3)
    b = pool.submit(bad, to_dev(zb, gpu), to_dev(wb, gpu), 3)
    recs = dict((r[0], r[2]) for r in pool.iterate())
    assert recs[b] == zm.ZM_REQ_FAILED and recs[a] == zm.ZM_REQ_LIVE
    pool.iterate(); pool.iterate()
    assert pool.query(a) == (zm.ZM_REQ_FINISHED, 3)
    got = fetch(pool, a, good, gpu)
    ref = solo(good, zg, wg, 3, gpu)
    assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1])
    pool.release(b)
    assert pool.query(b)[0] == zm.ZM_REQ_UNKNOWN


def test_pool_results_match_the_oracle(gpu):
    """Served results against the CPU oracle, not only against solo runs:
    a mix of four requests (even, odd and non-square sides, one of 64; FP64
    and FP32 pair forms; a budget that makes one wait) is served to the end,
    and every fetched state is compared with the oracle's own RK3
    trajectory: FP64 requests within 1e-12 (state) and 1e-9 (motion
    z - z0 and w), FP32 requests within 1e-5 on the motion and w."""
    import oracle
    import paper_2406_05490_amd as zm
    from zm_testutil import relerr
    reqs = []
    for (n1, n2), a, prec, steps, seed in (((64, 64), 0.6, zm.ZM_FP64, 3, 11),
                                           ((45, 45), 0.4, zm.ZM_FP32_PAIRS, 4, 12),
                                           ((40, 56), 0.8, zm.ZM_FP64, 2, 13),
                                           ((33, 30), 0.3, zm.ZM_FP32_PAIRS, 3, 14)):
        p = zm.Params(n1, n2, eps=1.0 / n1, atwood=a, gravity=1.0, dt=2e-3, precision=prec)
        z, w = rr.random_state(n1, n2, seed=seed, height=0.05)
        reqs.append((p, z, w, steps))
    sizes = sorted(zm.pool_request_bytes(p) for p, *_ in reqs)
    pool = zm.Pool(sizes[-1] + sizes[-2] + sizes[0])
    ids = [pool.submit(p, to_dev(z, gpu), to_dev(w, gpu), steps) for p, z, w, steps in reqs]
    index = {rid: i for i, rid in enumerate(ids)}
    results, live = {}, []
    for _ in range(50):
        recs = pool.iterate()
        if not recs and pool.stats().queued == 0:
            break
        live.append(len(recs))
        for rid, done, state, _ in recs:
            if state == zm.ZM_REQ_FINISHED:
                results[rid] = fetch(pool, rid, reqs[index[rid]][0], gpu)
                pool.release(rid)
    assert max(live) >= 2 and sorted(results) == sorted(ids)
    for rid, (p, z, w, steps) in zip(ids, reqs):
        P = oracle.Problem(p.n1, p.n2, eps=p.eps, atwood=p.atwood, gravity=p.gravity, dt=p.dt)
        zr, wr = oracle.rk3(P, z, w, steps)
        zg = results[rid][0].reshape(3, -1)
        wg = results[rid][1].reshape(2, -1)
        e_motion = relerr(zg - z, zr - z)
        e_w = relerr(wg - w, wr - w)
        if p.precision == zm.ZM_FP64:
            assert relerr(zg, zr) < 1e-12, (p.n1, p.n2)
            assert e_motion < 1e-9 and e_w < 1e-9, (p.n1, p.n2, e_motion, e_w)
        else:
            assert e_motion < 1e-5 and e_w < 1e-5, (p.n1, p.n2, e_motion, e_w)
    assert pool.stats().used_bytes == 0
