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


# --- w_t at sampled targets with the velocity in V handed in ----------------
# (the route the bench-size parity tests take: numpy's FFT velocity in, the
# oracle's V and difference stencil out)

@pytest.mark.parametrize("n1,n2,m1,m2,L1,L2", [(32, 32, 1, 0, 2.0, 2.0), (24, 24, 1, 3, 3.0, 1.5)])
def test_wt_sampled_flat_sheet_closed_form(n1, n2, m1, m2, L1, L2):
    """Flat sheet, w = grad cos(k.alpha) and the velocity written out by hand
    as -|k|/2 cos(k.alpha) e3: V = A |k|^2/4 cos(2 k.alpha), whose 5-point
    derivative is the closed form below (no velocity solver involved)."""
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
    kk = math.hypot(k1, k2)
    u = np.stack([0.0 * ph, 0.0 * ph, -0.5 * kk * np.cos(ph)])
    idx = np.array([0, 5, n1 - 1, n1 * n2 // 2 + 3, n1 * n2 - 1])
    wt = oracle.wt_sampled(P, z, w, u, idx)
    amp = A * kk * kk / 4.0
    ref1 = -amp * mod_wavenumber(2 * k1, h1) * np.sin(2 * ph[idx])
    ref2 = -amp * mod_wavenumber(2 * k2, h2) * np.sin(2 * ph[idx])
    scale = amp * max(abs(mod_wavenumber(2 * k1, h1)), abs(mod_wavenumber(2 * k2, h2)))
    assert np.max(np.abs(wt[0] - ref1)) < 1e-11 * scale
    assert np.max(np.abs(wt[1] - ref2)) < 1e-11 * scale


def test_wt_sampled_gravity_term_closed_form():
    """u = 0 and w = 0 leave V = -2 A g z3; with z3 = a cos(k alpha1) the
    5-point derivative is 2 A g a k~(k) sin(k alpha1)."""
    n, A, g, a = 32, 0.4, 2.5, 0.03
    P = prob(n, model=2, atwood=A, gravity=g)
    z, _ = rr.flat_state(n, n)
    h = 2.0 / n
    a1 = ((np.arange(n) * h)[None, :] + 0.0 * np.arange(n)[:, None]).ravel()
    k = 2 * math.pi * 2 / 2.0
    z[2] = a * np.cos(k * a1)
    w = np.zeros((2, n * n))
    idx = np.arange(0, n * n, 7)
    wt = oracle.wt_sampled(P, z, w, np.zeros((3, n * n)), idx)
    ref = 2.0 * A * g * a * mod_wavenumber(k, h) * np.sin(k * a1[idx])
    assert np.max(np.abs(wt[0] - ref)) < 1e-12 * 2.0 * A * g * a * k
    assert np.max(np.abs(wt[1])) < 1e-13 * 2.0 * A * g * a * k


@pytest.mark.parametrize("nu", [0.0, 2e-3])
def test_wt_sampled_reproduces_the_full_field_rhs(nu):
    """Fed the oracle's own low-order velocity, it returns the medium-order
    w_t of the full-field F bit for bit; fed the BR velocity, the high-order
    w_t of the sampled F."""
    n1, n2 = 16, 12
    z, w = rr.random_state(n1, n2, seed=7, height=0.1)
    kw = dict(atwood=0.6, gravity=1.1, nu=nu)
    Pm = prob(n1, n2, model=2, **kw)
    ulo, _ = oracle.rhs(prob(n1, n2, model=1, **kw), z, w)
    _, wm = oracle.rhs(Pm, z, w)
    idx = np.arange(n1 * n2)
    assert np.array_equal(oracle.wt_sampled(Pm, z, w, ulo, idx), wm)
    Ph = prob(n1, n2, model=0, **kw)
    sub = np.array([0, 3, n1 + 1, 77, n1 * n2 - 1])
    _, wh = oracle.rhs_sampled(Ph, z, w, sub)
    ubr = oracle.br_velocity(Ph, z, w)
    assert np.array_equal(oracle.wt_sampled(Ph, z, w, ubr, sub), wh)
    with pytest.raises(ValueError):
        oracle.wt_sampled(Pm, z, w, ulo, np.array([n1 * n2]))
