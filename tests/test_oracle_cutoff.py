"""Pins of the oracle's cutoff Birkhoff-Rott sum (CPU only).

The cutoff solver sums the desingularised kernel over the sources whose
nearest periodic image lies within a 3D distance rc of the target (the
paper's cutoff-based approximate integral calculation).  Checked against:
  * a flat sheet carrying a plane wave, where the sum over the lattice disc
    |rho| < rc has a closed form written out independently below;
  * a pure-Python brute force on tiny meshes;
  * mirror / sign / relabelling symmetries;
  * the exact all-pairs sum, which it must approach as rc grows.
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
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / np.max(np.abs(b)))


def disc_eigenvalue(n1, n2, k1, k2, eps, rc):
    """Flat sheet z = (a1, a2, 0), w = grad cos(k.a): the source strength is
    (-w2, w1, 0), (r x g)_3 = rho . w_j with rho = a_i - a_j, and the part of
    sin(k.a_j) odd in rho cancels over the symmetric disc, leaving
        u3 = lambda cos(k.a_i),
        lambda = -(h1 h2 / 4 pi) sum_{0 < |rho| < rc} (rho . k) sin(k . rho)
                 (|rho|^2 + eps^2)^(-3/2)."""
    h1, h2 = 2.0 / n1, 2.0 / n2
    m1 = np.arange(-n1, n1 + 1)
    m2 = np.arange(-n2, n2 + 1)
    R1, R2 = np.meshgrid(m1 * h1, m2 * h2, indexing="xy")
    rr2 = R1 * R1 + R2 * R2
    inside = rr2 < rc * rc
    # keep rc away from lattice distances so rounding cannot move a point
    assert np.min(np.abs(rr2 - rc * rc)) > 1e-9
    kr = k1 * R1 + k2 * R2
    terms = kr * np.sin(kr) * (rr2 + eps * eps) ** -1.5
    return -(h1 * h2) / (4 * math.pi) * float(np.sum(terms[inside]))


def mode_w(n1, n2, k1, k2):
    A1, A2 = rr.grid(n1, n2)
    s = np.sin(k1 * A1 + k2 * A2)
    mu = np.cos(k1 * A1 + k2 * A2)
    return np.stack([-k1 * s, -k2 * s]).reshape(2, -1), mu.ravel()


@pytest.mark.parametrize("n1,n2,k1,k2,rc", [
    (32, 32, math.pi, 0.0, 0.31), (32, 32, math.pi, 2 * math.pi, 0.52),
    (24, 40, 2 * math.pi, math.pi, 0.43), (16, 16, math.pi, -math.pi, 0.87),
])
def test_cutoff_flat_sheet_disc_closed_form(n1, n2, k1, k2, rc):
    eps = 1.0 / n1
    P = prob(n1, n2, eps=eps, cutoff=rc)
    z, _ = rr.flat_state(n1, n2)
    w, mu = mode_w(n1, n2, k1, k2)
    u = oracle.br_velocity(P, z, w)
    assert np.max(np.abs(u[:2])) < 1e-15
    lam = disc_eigenvalue(n1, n2, k1, k2, eps, rc)
    assert np.max(np.abs(u[2] - lam * mu)) < 1e-12 * abs(lam)


def brute_cutoff(n1, n2, z, gamma, eps, rc, L=2.0):
    """Pure-Python cutoff sum, nearest image per axis, straight loops."""
    N = n1 * n2
    h1, h2 = L / n1, L / n2
    coef = -(h1 * h2) / (4 * math.pi)
    u = np.zeros((3, N))
    for i in range(N):
        acc = [0.0, 0.0, 0.0]
        for j in range(N):
            d = [z[0][i] - z[0][j], z[1][i] - z[1][j], z[2][i] - z[2][j]]
            d[0] -= round(d[0] / L) * L
            d[1] -= round(d[1] / L) * L
            dd = d[0] ** 2 + d[1] ** 2 + d[2] ** 2
            if dd >= rc * rc:
                continue
            wgt = (dd + eps * eps) ** -1.5
            g = gamma[:, j]
            acc[0] += wgt * (d[1] * g[2] - d[2] * g[1])
            acc[1] += wgt * (d[2] * g[0] - d[0] * g[2])
            acc[2] += wgt * (d[0] * g[1] - d[1] * g[0])
        u[:, i] = [coef * a for a in acc]
    return u


@pytest.mark.parametrize("n1,n2,rc,seed", [(8, 8, 0.55, 0), (10, 6, 0.8, 1), (9, 12, 0.37, 2)])
def test_cutoff_matches_brute_force(n1, n2, rc, seed):
    eps = 0.5 * 2.0 / n1
    P = prob(n1, n2, eps=eps, cutoff=rc)
    z, w = rr.random_state(n1, n2, seed=seed, height=0.2)
    # drift across the seam so that images matter
    z[0] += 0.13
    _, _, gam, _ = oracle.surface(P, z, w)
    u = oracle.br_velocity(P, z, w)
    ref = brute_cutoff(n1, n2, z, gam, eps, rc)
    assert relerr(u, ref) < 1e-13


def test_cutoff_symmetries_bitwise():
    n = 16
    P = prob(n, cutoff=0.42)
    z, w = rr.random_state(n, n, seed=3, height=0.1)
    u = oracle.br_velocity(P, z, w)
    assert np.array_equal(oracle.br_velocity(P, z, -w), -u)
    zm = z.copy(); zm[2] = -zm[2]
    um = oracle.br_velocity(P, zm, w)
    assert np.array_equal(um[:2], -u[:2]) and np.array_equal(um[2], u[2])


def test_cutoff_relabelling_invariance():
    """Rolling the mesh index and re-basing x by the rolled cells changes
    nothing but the summation order."""
    n1, n2, s = 20, 16, 7
    P = prob(n1, n2, cutoff=0.5)
    z, w = rr.random_state(n1, n2, seed=4, height=0.1)
    u = oracle.br_velocity(P, z, w)
    Z = z.reshape(3, n2, n1); W = w.reshape(2, n2, n1)
    idx = (np.arange(n1) + s) % n1
    Zr = Z[:, :, idx].copy(); Wr = W[:, :, idx].copy()
    wrapped = np.arange(n1) + s >= n1
    Zr[0][:, wrapped] += 2.0
    ur = oracle.br_velocity(P, Zr.reshape(3, -1), Wr.reshape(2, -1))
    assert relerr(ur.reshape(3, n2, n1), u.reshape(3, n2, n1)[:, :, idx]) < 1e-13


def test_cutoff_tends_to_exact_sum():
    """The error against the exact all-pairs sum falls as rc grows (only the
    corners of the period cell beyond rc are missing at the largest rc)."""
    n = 24
    z, w = rr.random_state(n, n, seed=5, height=0.05)
    exact = oracle.br_velocity(prob(n), z, w)
    errs = [relerr(oracle.br_velocity(prob(n, cutoff=rc), z, w), exact)
            for rc in (0.2, 0.4, 0.6, 0.9)]
    assert all(a > b for a, b in zip(errs, errs[1:]))
    assert errs[-1] < 0.2 * errs[0]


def test_cutoff_rejects_bad_arguments():
    z, w = rr.random_state(8, 8, seed=6)
    for kw in ({"cutoff": 0.95}, {"cutoff": -0.1}, {"cutoff": 0.3, "images": 1}):
        with pytest.raises(ValueError):
            oracle.br_velocity(prob(8, **kw), z, w)


def test_cutoff_below_the_spacing_leaves_only_the_self_pair():
    """rc below every pair distance: only the self pair is inside, and it
    contributes exactly zero (r = 0), so u = 0 bit for bit."""
    n = 16
    z, w = rr.random_state(n, n, seed=21, height=0.05)
    P = oracle.Problem(n, n, eps=1.0 / n, cutoff=0.01)
    assert np.all(oracle.br_velocity(P, z, w) == 0.0)


@pytest.mark.parametrize("bump", [False, True])
def test_cutoff_boundary_is_strict(bump):
    """rc exactly two spacings on a flat mesh with h a power of two: the pairs
    exactly 2h apart have |r|^2 == rc^2 in binary and stay out (the strict
    inequality of the definition); one ulp more takes them in.  The closed
    form over the lattice disc tells the two apart (9 and 13 points)."""
    n = 32
    h = 2.0 / n
    rc = 2.0 * h
    if bump:
        rc = float(np.nextafter(rc, np.inf))
    eps = 1.0 / n
    k1, k2 = math.pi, 2 * math.pi
    P = prob(n, n, eps=eps, cutoff=rc)
    z, _ = rr.flat_state(n, n)
    w, mu = mode_w(n, n, k1, k2)
    u = oracle.br_velocity(P, z, w)
    m = np.arange(-n, n + 1)
    R1, R2 = np.meshgrid(m * h, m * h, indexing="xy")
    rr2 = R1 * R1 + R2 * R2
    inside = rr2 < rc * rc
    assert np.count_nonzero(inside) == (13 if bump else 9)
    kr = k1 * R1 + k2 * R2
    lam = -(h * h) / (4 * math.pi) * float(np.sum((kr * np.sin(kr) * (rr2 + eps * eps) ** -1.5)[inside]))
    assert np.max(np.abs(u[2] - lam * mu)) < 1e-12 * abs(lam)
