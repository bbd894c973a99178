"""Pins of the oracle's medium-order model (CPU only).

Reading: the medium-order model couples the two velocity solvers; the sheet
moves with the Birkhoff-Rott velocity (exact or cutoff) and the vorticity
law's Bernoulli potential takes the flat-sheet FFT velocity.  Checked
against:
  * a closed form on the flat sheet: with w = grad cos(k.alpha) the FFT
    velocity is exactly -|k|/2 cos(k.alpha) e3, so V = A |k|^2/4 cos(2 k.alpha)
    and w_t = -A |k|^2/4 k~(2k) sin(2 k.alpha), k~ the 5-point modified
    wavenumber; the BR velocity's eigenvalue differs from -|k|/2 by O(1e-3)
    at these meshes, so V built from it fails this pin;
  * its parts: z_t equals the high-order z_t and w_t the low-order w_t,
    bitwise, on random non-flat states (exact and cutoff BR);
  * the linear growth of a small single mode, which must be the high-order
    one (|u|^2 and q are quadratic).
"""
import math

import numpy as np
import pytest

import oracle
import rocket_rig as rr


def prob(n1, n2=None, **kw):
    n2 = n1 if n2 is None else n2
    kw.setdefault("eps", 0.5 * 2.0 / n1)
    return oracle.Problem(n1, n2, **kw)


def mod_wavenumber(k, h):
    return (8.0 * math.sin(k * h) - math.sin(2.0 * k * h)) / (6.0 * h)


@pytest.mark.parametrize("n1,n2,m1,m2,L1,L2", [(32, 32, 1, 0, 2.0, 2.0), (32, 16, 2, -1, 2.0, 2.0),
                                              (24, 24, 1, 3, 3.0, 1.5)])
def test_medium_flat_sheet_closed_form(n1, n2, m1, m2, L1, L2):
    A, g = 0.7, 1.3
    P = prob(n1, n2, model=2, atwood=A, gravity=g, period1=L1, period2=L2)
    z, _ = rr.flat_state(n1, n2)
    z[0] *= L1 / 2.0
    z[1] *= L2 / 2.0
    h1, h2 = L1 / n1, L2 / n2
    a1 = (np.arange(n1) * h1)[None, :] + 0.0 * np.arange(n2)[:, None]
    a2 = (np.arange(n2) * h2)[:, None] + 0.0 * np.arange(n1)[None, :]
    k1, k2 = 2 * math.pi * m1 / L1, 2 * math.pi * m2 / L2
    ph = (k1 * a1 + k2 * a2).ravel()
    w = np.stack([-k1 * np.sin(ph), -k2 * np.sin(ph)])
    zt, wt = oracle.rhs(P, z, w)
    kk = math.hypot(k1, k2)
    amp = A * kk * kk / 4.0
    ref1 = -amp * mod_wavenumber(2 * k1, h1) * np.sin(2 * ph)
    ref2 = -amp * mod_wavenumber(2 * k2, h2) * np.sin(2 * ph)
    scale = amp * max(abs(mod_wavenumber(2 * k1, h1)), abs(mod_wavenumber(2 * k2, h2)))
    assert np.max(np.abs(wt[0] - ref1)) < 1e-11 * scale
    assert np.max(np.abs(wt[1] - ref2)) < 1e-11 * scale
    # the sheet moves with the BR velocity: flat-sheet eigenvector, tangential part 0
    assert np.max(np.abs(zt[:2])) == 0.0
    lam = float(zt[2] @ np.cos(ph) / (np.cos(ph) @ np.cos(ph)))
    assert abs(lam + kk / 2.0) > 1e-4 * kk          # not the FFT symbol
    assert np.max(np.abs(zt[2] - lam * np.cos(ph))) < 1e-12 * kk


@pytest.mark.parametrize("cutoff", [0.0, 0.4])
def test_medium_is_high_z_and_low_w(cutoff):
    n1, n2 = 16, 8
    z, w = rr.random_state(n1, n2, seed=3, height=0.1)
    kw = dict(atwood=0.6, gravity=1.1, nu=1e-3, cutoff=cutoff)
    zm_, wm = oracle.rhs(prob(n1, n2, model=2, **kw), z, w)
    zh, _ = oracle.rhs(prob(n1, n2, model=0, **kw), z, w)
    kl = dict(kw, cutoff=0.0)
    _, wl = oracle.rhs(prob(n1, n2, model=1, **kl), z, w)
    assert np.array_equal(zm_, zh)
    assert np.array_equal(wm, wl)
    # the two velocities really differ on this state
    zl, _ = oracle.rhs(prob(n1, n2, model=1, **kl), z, w)
    assert np.max(np.abs(zl - zh)) > 1e-3 * np.max(np.abs(zh))


def test_medium_linear_growth_is_high_order():
    n = 16
    z, _ = rr.single_mode(n, n, 1e-6)
    w = np.zeros((2, n * n))
    kw = dict(dt=5e-3, atwood=0.5, gravity=1.0)
    zm_, wm = oracle.rk3(prob(n, model=2, **kw), z, w, 20)
    zh, wh = oracle.rk3(prob(n, model=0, **kw), z, w, 20)
    assert np.max(np.abs(zm_[2] - zh[2])) < 1e-6 * np.max(np.abs(zh[2]))
    assert np.max(np.abs(wm - wh)) < 1e-6 * np.max(np.abs(wh))


def test_medium_rejects_free_sheet_and_sampling():
    z, w = rr.random_state(8, 8, seed=5)
    with pytest.raises(ValueError):
        oracle.rhs(prob(8, model=2, boundary=1), z, w)
    with pytest.raises(ValueError):
        oracle.rhs_sampled(prob(8, model=2), z, w, np.array([0, 5]))
