"""Pins of the CPU oracle against closed forms, physics and invariants.

Nothing here compares the oracle with itself re-typed: each expected value is
a closed form (finite-difference symbols, the RK3 stability polynomial, the
flat-sheet Birkhoff-Rott eigenvalue -|k|/2, the Rayleigh-Taylor rate
sqrt(A g |k|), the Kelvin-Helmholtz rate |k| c / 2) or an exact symmetry of
the model.  A plausible slip in the oracle -- a sign, a dropped term, a
transposed operand, an unsplit periodic tie -- fails at least one of these.
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


def relerr(a, b):
    """Normwise: max |a - b| / max |b|."""
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / np.max(np.abs(b)))


def mode_w(n1, n2, k1, k2, amp=1.0):
    """w = grad(mu) analytic for mu = amp cos(k1 x + k2 y)."""
    A1, A2 = rr.grid(n1, n2)
    s = np.sin(k1 * A1 + k2 * A2)
    mu = amp * np.cos(k1 * A1 + k2 * A2)
    return np.stack([-amp * k1 * s, -amp * k2 * s]).reshape(2, -1), mu.ravel()


# --------------------------------------------------------------------------
# finite differences (tangents, Laplacian)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("n1,n2", [(16, 16), (24, 40), (33, 17)])
def test_fd_modified_wavenumber(n1, n2):
    """D cos(k a) = -k~ sin(k a), k~ = (8 sin kh - sin 2kh) / (6h); the
    second difference has symbol (-2 cos 2kh + 32 cos kh - 30) / (12 h^2)."""
    P = prob(n1, n2)
    A1, A2 = rr.grid(n1, n2)
    h1, h2 = 2.0 / n1, 2.0 / n2
    k1, k2 = 3 * math.pi, 2 * math.pi
    z, _ = rr.flat_state(n1, n2)
    f = np.cos(k1 * A1) * np.cos(k2 * A2)
    z[2] = f.ravel()
    t1, t2 = oracle.tangents(P, z)
    kt1 = (8 * math.sin(k1 * h1) - math.sin(2 * k1 * h1)) / (6 * h1)
    kt2 = (8 * math.sin(k2 * h2) - math.sin(2 * k2 * h2)) / (6 * h2)
    e1 = -kt1 * np.sin(k1 * A1) * np.cos(k2 * A2)
    e2 = -kt2 * np.cos(k1 * A1) * np.sin(k2 * A2)
    assert np.max(np.abs(t1[2] - e1.ravel())) < 1e-12 * kt1
    assert np.max(np.abs(t2[2] - e2.ravel())) < 1e-12 * kt2
    lap = oracle.laplacian(P, f.ravel())
    s1 = (-2 * math.cos(2 * k1 * h1) + 32 * math.cos(k1 * h1) - 30) / (12 * h1 * h1)
    s2 = (-2 * math.cos(2 * k2 * h2) + 32 * math.cos(k2 * h2) - 30) / (12 * h2 * h2)
    assert np.max(np.abs(lap - (s1 + s2) * f.ravel())) < 1e-10 * abs(s1 + s2)


@pytest.mark.parametrize("n1,n2", [(16, 16), (12, 20), (9, 11)])
def test_fd_flat_grid_tangents(n1, n2):
    """On the flat grid T1 = e1 and T2 = e2 to a few ulp, including across
    the seam (the periodic coordinate correction)."""
    P = prob(n1, n2)
    z, _ = rr.flat_state(n1, n2)
    t1, t2 = oracle.tangents(P, z)
    ulp = np.finfo(np.float64).eps
    assert np.max(np.abs(t1[0] - 1.0)) <= 8 * ulp
    assert np.max(np.abs(t2[1] - 1.0)) <= 8 * ulp
    assert np.all(t1[1] == 0) and np.all(t1[2] == 0)
    assert np.all(t2[0] == 0) and np.all(t2[2] == 0)


def test_q_is_inverse_metric_contraction():
    """q = |gamma|^2 / |T1 x T2|^2 equals g^{ab} w_a w_b (the squared surface
    gradient of the potential jump), with g_ab = T_a . T_b."""
    n = 20
    P = prob(n)
    z, w = rr.random_state(n, n, seed=5, height=0.2)
    t1, t2, g, q = oracle.surface(P, z, w)
    g11 = np.sum(t1 * t1, 0); g22 = np.sum(t2 * t2, 0); g12 = np.sum(t1 * t2, 0)
    det = g11 * g22 - g12 * g12
    expect = (g22 * w[0] ** 2 - 2 * g12 * w[0] * w[1] + g11 * w[1] ** 2) / det
    assert relerr(q, expect) < 1e-12
    # gamma is tangent to the surface and orthogonal to grad(mu)'s dual:
    nrm = np.cross(t1.T, t2.T).T
    assert np.max(np.abs(np.sum(g * nrm, 0))) < 1e-12 * np.max(np.abs(g))


# --------------------------------------------------------------------------
# Birkhoff-Rott velocity
# --------------------------------------------------------------------------

def test_rest_state_bitwise():
    """Flat interface, zero vorticity: u = 0 exactly, w_t = 0 exactly; z3 and w
    stay exactly zero over steps, x/y move by RK3 rounding only."""
    n = 16
    P = prob(n, atwood=0.5, gravity=1.0, dt=1e-2)
    z, w = rr.flat_state(n, n)
    u = oracle.br_velocity(P, z, w)
    assert np.all(u == 0.0)
    zt, wt = oracle.rhs(P, z, w)
    assert np.all(zt == 0.0) and np.all(wt == 0.0)
    z1, w1 = oracle.rk3(P, z, w, 5)
    assert np.all(z1[2] == 0.0) and np.all(w1 == 0.0)
    assert np.max(np.abs(z1[:2] - z[:2])) <= 5 * 2 * np.finfo(np.float64).eps


def lattice_eigenvalue(k1, k2, n1, n2, eps, kt=None, M=12):
    """Closed form of the flat-sheet BR eigenvalue summed over all periodic
    images.  The desingularised kernel (r^2 + eps^2)^(-3/2) has the 2D
    Fourier transform 2 pi exp(-|q| eps) / eps, so a plane wave mu =
    cos(k.a) with w = grad mu gives u3 = -(|k|/2) exp(-|k| eps) mu in the
    continuum; on the lattice h1 Z x h2 Z the Poisson summation formula adds
    the aliases q_m = k + 2 pi (m1/h1, m2/h2):
        lambda = sum_m -(1/2) (kt . q_m) / |q_m| exp(-|q_m| eps).
    kt replaces k in the source strength when w is a finite-difference
    gradient (modified wavenumbers)."""
    h1, h2 = 2.0 / n1, 2.0 / n2
    kt = (k1, k2) if kt is None else kt
    lam = 0.0
    for m1 in range(-M, M + 1):
        for m2 in range(-M, M + 1):
            q1 = k1 + 2 * math.pi * m1 / h1
            q2 = k2 + 2 * math.pi * m2 / h2
            qq = math.hypot(q1, q2)
            lam += -0.5 * (kt[0] * q1 + kt[1] * q2) / qq * math.exp(-qq * eps)
    return lam


def flat_lambda(n1, n2, k1, k2, images, eps=None):
    P = prob(n1, n2, images=images) if eps is None else prob(n1, n2, images=images, eps=eps)
    z, _ = rr.flat_state(n1, n2)
    w, mu = mode_w(n1, n2, k1, k2)
    u = oracle.br_velocity(P, z, w)
    return float(u[2] @ mu / (mu @ mu)), u, mu


@pytest.mark.parametrize("n1,n2,k1,k2", [(32, 32, math.pi, 0.0), (32, 32, math.pi, 2 * math.pi),
                                         (24, 36, 2 * math.pi, math.pi), (15, 9, math.pi, math.pi)])
def test_flat_sheet_eigenvector(n1, n2, k1, k2):
    """Flat sheet, w = grad cos(k.a): tangential u = 0 exactly and u3 is a
    multiple of cos(k.a), of the sign and size of -|k|/2 (within the
    desingularisation's damping and the one-cell truncation)."""
    lam, u, mu = flat_lambda(n1, n2, k1, k2, 0)
    assert np.all(u[0] == 0.0) and np.all(u[1] == 0.0)
    assert np.max(np.abs(u[2] - lam * mu)) < 1e-13 * abs(lam)
    ratio = lam / (-math.hypot(k1, k2) / 2)
    assert 0.6 < ratio < 1.15


@pytest.mark.parametrize("n1,n2,k1,k2", [(16, 16, math.pi, 0.0), (16, 16, math.pi, 2 * math.pi),
                                         (12, 20, 2 * math.pi, math.pi), (10, 14, math.pi, -math.pi)])
def test_flat_sheet_lattice_sum_closed_form(n1, n2, k1, k2):
    """As the image layers K grow, the eigenvalue tends to the Poisson-sum
    closed form; the square truncation error decays like 1/(2K+1), so a
    Richardson step over K = 8, 16 leaves about 1e-5.  This pins the sign,
    the h1 h2 / 4 pi normalisation, the eps placement, the cross-product
    orientation and the source strength w1 T2 - w2 T1."""
    exact = lattice_eigenvalue(k1, k2, n1, n2, eps=1.0 / n1)
    l8 = flat_lambda(n1, n2, k1, k2, 8)[0]
    l16 = flat_lambda(n1, n2, k1, k2, 16)[0]
    x8, x16 = 1.0 / 17, 1.0 / 33
    extrap = (l16 * x8 - l8 * x16) / (x8 - x16)
    assert abs(extrap / exact - 1) < 2e-4
    assert abs(l16 / exact - 1) < 0.02


def test_flat_sheet_lowest_mode_value():
    """k = (pi, 0) at N = 32, K = 0, eps = h/2: lambda within 0.5% of -pi/2.
    (A transposed source strength w1 T1 - w2 T2 gives 0 here; a wrong sign
    or a 2 pi normalisation is off by 100%.)"""
    lam = flat_lambda(32, 32, math.pi, 0.0, 0)[0]
    assert abs(lam / (-math.pi / 2) - 1) < 0.005


def test_vorticity_sign_flip_bitwise():
    n = 16
    P = prob(n)
    z, w = rr.random_state(n, n, seed=1, height=0.1)
    u = oracle.br_velocity(P, z, w)
    um = oracle.br_velocity(P, z, -w)
    assert np.array_equal(um, -u)


def test_vertical_mirror_bitwise():
    """z3 -> -z3 (w fixed) maps (u1,u2,u3) -> (-u1,-u2,u3); adding w -> -w
    gives (u1,u2,-u3)."""
    n = 16
    P = prob(n)
    z, w = rr.random_state(n, n, seed=2, height=0.1)
    u = oracle.br_velocity(P, z, w)
    zm = z.copy(); zm[2] = -zm[2]
    um = oracle.br_velocity(P, zm, w)
    assert np.array_equal(um[0], -u[0]) and np.array_equal(um[1], -u[1])
    assert np.array_equal(um[2], u[2])
    umm = oracle.br_velocity(P, zm, -w)
    assert np.array_equal(umm[:2], u[:2]) and np.array_equal(umm[2], -u[2])


def roll_axis1(z, w, n1, n2, s):
    """Relabel mesh point i1 -> i1 + s (periodic), keeping x continuous."""
    Z = z.reshape(3, n2, n1).copy(); W = w.reshape(2, n2, n1).copy()
    idx = (np.arange(n1) + s) % n1
    wraps = (np.arange(n1) + s) // n1
    Zr = Z[:, :, idx]; Wr = W[:, :, idx]
    Zr[0] = Zr[0] + wraps[None, :] * 2.0
    return Zr.reshape(3, -1), Wr.reshape(2, -1), idx


def roll_axis2(z, w, n1, n2, s):
    Z = z.reshape(3, n2, n1).copy(); W = w.reshape(2, n2, n1).copy()
    idx = (np.arange(n2) + s) % n2
    wraps = (np.arange(n2) + s) // n2
    Zr = Z[:, idx, :]; Wr = W[:, idx, :]
    Zr[1] = Zr[1] + wraps[:, None] * 2.0
    return Zr.reshape(3, -1), Wr.reshape(2, -1), idx


@pytest.mark.parametrize("n1,n2", [(16, 16), (15, 12)])
def test_periodic_translation(n1, n2):
    """Relabelling the periodic mesh (cyclic roll of the index, x and y kept
    continuous) rolls the velocity: the image rule and the seam correction
    depend on index offsets only."""
    P = prob(n1, n2)
    z, w = rr.random_state(n1, n2, seed=3, height=0.1)
    u = oracle.br_velocity(P, z, w).reshape(3, n2, n1)
    zr, wr, idx = roll_axis1(z, w, n1, n2, 5)
    ur = oracle.br_velocity(P, zr, wr).reshape(3, n2, n1)
    assert relerr(ur, u[:, :, idx]) < 1e-13
    zr, wr, idx = roll_axis2(z, w, n1, n2, 7)
    ur = oracle.br_velocity(P, zr, wr).reshape(3, n2, n1)
    assert relerr(ur, u[:, idx, :]) < 1e-13


@pytest.mark.parametrize("n1,n2", [(16, 16), (16, 13), (15, 15)])
def test_mirror_x(n1, n2):
    """i1 -> -i1 mod n1, z1 -> -z1, w1 -> -w1 maps u1 -> -u1 with u2, u3
    mirrored.  With even n1 this holds only if the tie at |o| = n1/2 is
    split between both images."""
    P = prob(n1, n2)
    z, w = rr.random_state(n1, n2, seed=4, height=0.1)
    u = oracle.br_velocity(P, z, w).reshape(3, n2, n1)
    Z = z.reshape(3, n2, n1); W = w.reshape(2, n2, n1)
    idx = (-np.arange(n1)) % n1
    Zm = Z[:, :, idx].copy(); Wm = W[:, :, idx].copy()
    Zm[0] = -Zm[0]
    Zm[0][:, 1:] = Zm[0][:, 1:] + 2.0     # keep x continuous and increasing
    Wm[0] = -Wm[0]
    um = oracle.br_velocity(P, Zm.reshape(3, -1), Wm.reshape(2, -1)).reshape(3, n2, n1)
    expect = u[:, :, idx].copy()
    expect[0] = -expect[0]
    assert relerr(um, expect) < 1e-13


def test_rigid_translation():
    n = 16
    P = prob(n)
    z, w = rr.random_state(n, n, seed=7, height=0.1)
    u = oracle.br_velocity(P, z, w)
    zt = z + np.array([0.3, -0.7, 0.2])[:, None]
    ut = oracle.br_velocity(P, zt, w)
    assert relerr(ut, u) < 1e-13


def test_axis_swap():
    """Swapping the two mesh axes (and x<->y, w1<->w2) swaps u1 and u2."""
    n = 12
    P = prob(n)
    z, w = rr.random_state(n, n, seed=8, height=0.1)
    u = oracle.br_velocity(P, z, w).reshape(3, n, n)
    Z = z.reshape(3, n, n); W = w.reshape(2, n, n)
    Zs = np.stack([Z[1].T, Z[0].T, Z[2].T]); Ws = np.stack([W[1].T, W[0].T])
    us = oracle.br_velocity(P, Zs.reshape(3, -1), Ws.reshape(2, -1)).reshape(3, n, n)
    expect = np.stack([u[1].T, u[0].T, u[2].T])
    assert relerr(us, expect) < 1e-13


def test_image_layers_converge():
    """Extra image layers K converge (the periodic lattice sum of the flat
    sheet eigenvalue approaches -|k|/2 from the K = 0 truncation)."""
    n = 16
    z, _ = rr.flat_state(n, n)
    w, mu = mode_w(n, n, math.pi, 0.0)
    lams = []
    for K in (0, 1, 2):
        P = prob(n, images=K)
        u = oracle.br_velocity(P, z, w)
        lams.append(float(u[2] @ mu / (mu @ mu)))
    d1 = abs(lams[1] - lams[0]); d2 = abs(lams[2] - lams[1])
    assert d2 < d1


def test_sampled_targets_match_full():
    n1, n2 = 12, 10
    P = prob(n1, n2)
    z, w = rr.random_state(n1, n2, seed=9, height=0.1)
    u = oracle.br_velocity(P, z, w)
    t = np.array([0, 5, 37, 119, 64])
    us = oracle.br_velocity(P, z, w, targets=t)
    assert np.array_equal(us, u[:, t])
    zt, wt = oracle.rhs(P, z, w)
    zs, ws = oracle.rhs_sampled(P, z, w, t)
    assert np.array_equal(zs, zt[:, t])
    assert np.max(np.abs(ws - wt[:, t])) <= 1e-15 * np.max(np.abs(wt))


def test_thread_count_independent():
    n = 16
    P = prob(n)
    z, w = rr.random_state(n, n, seed=10, height=0.1)
    assert np.array_equal(oracle.br_velocity(P, z, w, threads=1),
                          oracle.br_velocity(P, z, w, threads=3))


# --------------------------------------------------------------------------
# growth rates: RT (pins BR sign/normalisation + A g term + RK3) and KH
# (pins the 3D geometry of the kernel: the r3 component and marker motion)
# --------------------------------------------------------------------------

def rt_sigma_d(n, atwood=0.5, g=1.0, images=0):
    """sigma_d^2 from one application of the discrete linear operator:
    w = -2 A g D(z3) for z3 = cos(pi x) cos(pi y) on the flat sheet, then the
    normal BR velocity per unit z3."""
    P = prob(n, images=images)
    z, _ = rr.flat_state(n, n)
    A1, A2 = rr.grid(n, n)
    f = (np.cos(math.pi * A1) * np.cos(math.pi * A2)).ravel()
    zz = z.copy(); zz[2] = f
    t1, t2 = oracle.tangents(P, zz)
    w = np.stack([-2 * atwood * g * t1[2], -2 * atwood * g * t2[2]])
    u = oracle.br_velocity(P, z, w)
    return math.sqrt(float(u[2] @ f / (f @ f)))


def test_rt_rate_approaches_sqrt_agk():
    """sigma_d -> sqrt(A g |k|) (the linear Rayleigh-Taylor rate), |k| =
    pi sqrt(2): within 3% from N = 64 on, and increasing with N."""
    exact = math.sqrt(0.5 * 1.0 * math.pi * math.sqrt(2.0))
    s32, s64 = rt_sigma_d(32), rt_sigma_d(64)
    assert s32 < s64 < exact * 1.03
    assert abs(s64 / exact - 1) < 0.03


def test_rt_rate_lattice_closed_form():
    """With many image layers the discrete RT rate matches the closed form
    sigma^2 = -2 A g lambda(k; k~), where k~ are the fourth-order modified
    wavenumbers of D applied to z3 (pins the A g term, the FD gradient of
    V and the BR normal velocity together)."""
    n, A, g = 16, 0.5, 1.0
    h = 2.0 / n
    kt = (8 * math.sin(math.pi * h) - math.sin(2 * math.pi * h)) / (6 * h)
    lam = lattice_eigenvalue(math.pi, math.pi, n, n, eps=h / 2, kt=(kt, kt))
    exact = math.sqrt(-2 * A * g * lam)
    s8, s16 = rt_sigma_d(n, images=8) ** 2, rt_sigma_d(n, images=16) ** 2
    x8, x16 = 1.0 / 17, 1.0 / 33
    extrap = math.sqrt((s16 * x8 - s8 * x16) / (x8 - x16))
    assert abs(extrap / exact - 1) < 2e-4


def test_rt_linear_growth_follows_rk3_polynomial():
    """Small single mode from rest: after n SSP-RK3 steps the amplitude is
    a (R(s dt)^n + R(-s dt)^n) / 2 with R(x) = 1 + x + x^2/2 + x^3/6 (the RK3
    stability polynomial) and s = sigma_d; this pins the three stage
    combinations and the linear terms z_t = u, w_t = D(-2 A g z3)."""
    n, a, dt, steps = 16, 1e-6, 5e-3, 200
    P = prob(n, atwood=0.5, gravity=1.0, dt=dt)
    s = rt_sigma_d(n)
    z, w = rr.single_mode(n, n, a)
    z1, _ = oracle.rk3(P, z, w, steps)
    A1, A2 = rr.grid(n, n)
    f = (np.cos(math.pi * A1) * np.cos(math.pi * A2)).ravel()
    amp = float(z1[2] @ f / (f @ f))
    R = lambda x: 1 + x + x * x / 2 + x ** 3 / 6
    pred = a * (R(s * dt) ** steps + R(-s * dt) ** steps) / 2
    assert abs(amp / pred - 1) < 1e-6
    # and it is the cosh growth to RK3 truncation accuracy
    assert abs(amp / (a * math.cosh(s * dt * steps)) - 1) < 1e-6


def kh_lattice_symbols(k1, k2, n1, n2, eps, c=1.0, M=12):
    """Closed forms of the two linear Kelvin-Helmholtz operators of a flat
    sheet with uniform shear w = (c, 0) (gamma = c e2), summed over all
    periodic images (Poisson summation, kernel transform G^(q) = 2 pi
    exp(-|q| eps) / eps):
      z3 = cos(k.a)  ->  u1 = s1 cos(k.a),  s1 = c/(4 pi) sum_m [G^(Q_m) - G^(Q_m + k)]
      z1 += cos(k.a) ->  u3 = s3 cos(k.a),  s3 = -c/(4 pi) sum_m [H(Q_m) - H(Q_m + k)]
    with H(q) = 2 pi q1^2 / |q| exp(-|q| eps) the transform of d/dr1 (r1 G).
    In the continuum (m = 0, eps -> 0) both tend to c |k| / 2 for k along
    x, giving the classical rate |k| c / 2."""
    h1, h2 = 2.0 / n1, 2.0 / n2
    G = lambda q: 2 * math.pi * math.exp(-q * eps) / eps
    H = lambda q1, q: 0.0 if q == 0.0 else 2 * math.pi * (q1 * q1 / q) * math.exp(-q * eps)
    s1 = s3 = 0.0
    for m1 in range(-M, M + 1):
        for m2 in range(-M, M + 1):
            Q1, Q2 = 2 * math.pi * m1 / h1, 2 * math.pi * m2 / h2
            q0, qk = math.hypot(Q1, Q2), math.hypot(Q1 + k1, Q2 + k2)
            s1 += G(q0) - G(qk)
            s3 += H(Q1, q0) - H(Q1 + k1, qk)
    return c / (4 * math.pi) * s1, -c / (4 * math.pi) * s3


def kh_measured(n1, n2, k1, k2, images, a=1e-7, c=1.0):
    P = prob(n1, n2, images=images)
    A1, A2 = rr.grid(n1, n2)
    f = np.cos(k1 * A1 + k2 * A2).ravel()
    z, _ = rr.flat_state(n1, n2)
    w = np.stack([np.full(n1 * n2, c), np.zeros(n1 * n2)])
    z3 = z.copy(); z3[2] = a * f
    s1 = float(oracle.br_velocity(P, z3, w)[0] @ f / (f @ f)) / a
    zx = z.copy(); zx[0] = zx[0] + a * f
    s3 = float(oracle.br_velocity(P, zx, w)[2] @ f / (f @ f)) / a
    return s1, s3


@pytest.mark.parametrize("n1,n2,k1,k2", [(16, 16, math.pi, 0.0), (12, 20, 2 * math.pi, 0.0), (14, 10, math.pi, 0.0)])
def test_kh_operators_lattice_closed_form(n1, n2, k1, k2):
    """The 3D geometry of the kernel: a vertical displacement induces
    horizontal velocity through the r3 component (s1), a horizontal marker
    displacement induces vertical velocity (s3).  Both match their
    image-summed closed forms after a Richardson step over K = 8, 16.  The
    modes are independent of alpha_2, so T2 = e2 and the source strength
    stays c e2 (the closed form assumes that)."""
    e1, e3 = kh_lattice_symbols(k1, k2, n1, n2, eps=1.0 / n1)
    a8 = kh_measured(n1, n2, k1, k2, 8)
    a16 = kh_measured(n1, n2, k1, k2, 16)
    x8, x16 = 1.0 / 17, 1.0 / 33
    for m8, m16, exact in ((a8[0], a16[0], e1), (a8[1], a16[1], e3)):
        extrap = (m16 * x8 - m8 * x16) / (x8 - x16)
        assert abs(extrap / exact - 1) < 3e-4


def test_kh_linear_growth():
    """Equal densities (A = 0), uniform shear, small z3 = a cos(pi x): the
    vorticity stays frozen exactly and the amplitude follows the RK3
    polynomial with sigma^2 = s1 s3 (the two operators measured at K = 0)."""
    n, a, dt, steps = 16, 1e-6, 2e-2, 50
    s1, s3 = kh_measured(n, n, math.pi, 0.0, 0)
    sigma = math.sqrt(s1 * s3)
    P = prob(n, atwood=0.0, gravity=1.0, dt=dt)
    z, _ = rr.flat_state(n, n)
    A1, _ = rr.grid(n, n)
    f = np.cos(math.pi * A1).ravel()
    z[2] = a * f
    w = np.stack([np.ones(n * n), np.zeros(n * n)])
    z1, w1 = oracle.rk3(P, z, w, steps)
    assert np.array_equal(w1, w)
    amp = float(z1[2] @ f / (f @ f))
    R = lambda x: 1 + x + x * x / 2 + x ** 3 / 6
    pred = a * (R(sigma * dt) ** steps + R(-sigma * dt) ** steps) / 2
    assert abs(amp / pred - 1) < 1e-5


def test_atwood_zero_freezes_vorticity():
    n = 12
    P = prob(n, atwood=0.0, dt=1e-2)
    z, w = rr.random_state(n, n, seed=11, height=0.1)
    zt, wt = oracle.rhs(P, z, w)
    assert np.all(wt == 0.0)
    z1, w1 = oracle.rk3(P, z, w, 3)
    # w_t = 0 exactly; the RK3 convex combination 1/3 w + 2/3 w may round
    # by an ulp per step
    assert np.all(np.abs(w1 - w) <= 3 * 2 * np.finfo(np.float64).eps * np.abs(w))
    assert not np.array_equal(z1, z)


def test_whole_problem_mirror_bitwise():
    """(z3, w, A, g) -> (-z3, -w, -A, -g) maps the trajectory to
    (z1, z2, -z3, -w) exactly."""
    n = 10
    P = prob(n, atwood=0.5, gravity=1.0, dt=1e-2)
    Pm = prob(n, atwood=-0.5, gravity=-1.0, dt=1e-2)
    z, w = rr.random_state(n, n, seed=12, height=0.1)
    za, wa = oracle.rk3(P, z, w, 3)
    zm = z.copy(); zm[2] = -zm[2]
    zb, wb = oracle.rk3(Pm, zm, -w, 3)
    assert np.array_equal(zb[:2], za[:2]) and np.array_equal(zb[2], -za[2])
    assert np.array_equal(wb, -wa)


def test_time_convergence_order3():
    """Self-convergence of the full nonlinear model: halving dt cuts the
    difference by about 2^3."""
    n, T = 12, 0.2
    z, w = rr.random_state(n, n, seed=13, height=0.1)
    res = []
    for k in range(4):
        dt = 0.02 / 2 ** k
        P = prob(n, atwood=0.5, gravity=1.0, dt=dt)
        res.append(np.concatenate(oracle.rk3(P, z, w, int(round(T / dt)))))
    e1 = np.max(np.abs(res[0] - res[1])); e2 = np.max(np.abs(res[1] - res[2]))
    e3 = np.max(np.abs(res[2] - res[3]))
    assert 6.0 < e1 / e2 < 10.0
    assert 6.0 < e2 / e3 < 10.0
