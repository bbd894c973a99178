"""Seeded input generators: deterministic, in range, shaped as documented."""
import numpy as np

import rocket_rig as rr


def test_generators_deterministic():
    a = rr.multi_mode(32, 24, 8, seed=1)
    b = rr.multi_mode(32, 24, 8, seed=1)
    assert np.array_equal(a[0], b[0]) and a[0].shape == (3, 32 * 24)
    assert not np.array_equal(a[0], rr.multi_mode(32, 24, 8, seed=2)[0])
    assert np.array_equal(rr.synthetic_vorticity(16, 16, 3), rr.synthetic_vorticity(16, 16, 3))


def test_grid_and_noise():
    z, w = rr.single_mode(16, 8, 0.0, noise=1e-4, seed=0)
    assert np.all(np.abs(z[2]) <= 1e-4) and np.all(w == 0)
    A1, A2 = rr.grid(16, 8)
    assert A1[0, 0] == -1.0 and np.isclose(A1[0, 1] - A1[0, 0], 2 / 16)
    assert np.array_equal(z[0], A1.ravel()) and np.array_equal(z[1], A2.ravel())


def test_ensemble_and_requests():
    e = rr.ensemble(64, seed=3)
    assert len(e) == 64 and all(m.n in rr.ENSEMBLE_SIDES for m in e)
    assert all(0.1 <= m.atwood <= 0.9 and 0.01 <= m.amplitude <= 0.1 for m in e)
    assert [m.n for m in e] == [m.n for m in rr.ensemble(64, seed=3)]
    r = rr.request_stream(200, rate=5.0, seed=4)
    assert all(64 <= m.n <= 512 and m.n % 8 == 0 for m in r)
    assert all(100 <= m.steps <= 1000 for m in r)
    t = [m.arrival for m in r]
    assert all(b > a for a, b in zip(t, t[1:]))
    assert 20 < t[-1] < 60      # 200 arrivals at 5/s


def test_sample_targets():
    t = rr.sample_targets(1000, 50, seed=1)
    assert len(set(t.tolist())) == 50 and np.all(np.diff(t) > 0) and t.max() < 1000
