"""Pins of the oracle's free (non-periodic) boundary (CPU only).

A non-periodic sheet gets its stencil values beyond the edges by cubic
extrapolation into the boundary cells, and its BR sum has no periodic
images.  Checked against:
  * polynomials the extrapolated stencils must differentiate exactly;
  * a pure-Python free-space brute force;
  * rigid translation (any vector) and mirror symmetry through x = const,
    which also exercises the two ends' ghost formulas;
  * with a cutoff: a free-space brute force over the pairs within rc, and
    the exact free sum once rc exceeds the sheet's diameter.
"""
import math

import numpy as np
import pytest

import oracle
import rocket_rig as rr


def prob(n1, n2=None, **kw):
    n2 = n1 if n2 is None else n2
    kw.setdefault("eps", 0.5 * 2.0 / n1)
    return oracle.Problem(n1, n2, boundary=1, **kw)


def relerr(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / np.max(np.abs(b)))


@pytest.mark.parametrize("n1,n2", [(8, 8), (12, 9), (16, 24)])
def test_free_stencils_exact_on_cubics(n1, n2):
    A1, A2 = rr.grid(n1, n2)
    c = 0.3 + 0.7 * A1 - 0.5 * A1 ** 2 + 0.25 * A1 ** 3
    d = -0.2 + 0.4 * A2 + 0.3 * A2 ** 2 - 0.6 * A2 ** 3
    z = np.stack([A1.ravel(), A2.ravel(), (c * d).ravel()])
    P = prob(n1, n2)
    t1, t2 = oracle.tangents(P, z)
    dc = 0.7 - 1.0 * A1 + 0.75 * A1 ** 2
    dd = 0.4 + 0.6 * A2 - 1.8 * A2 ** 2
    assert np.max(np.abs(t1[2] - (dc * d).ravel())) < 1e-12
    assert np.max(np.abs(t2[2] - (c * dd).ravel())) < 1e-12
    assert np.max(np.abs(t1[0] - 1.0)) < 1e-13 and np.max(np.abs(t2[1] - 1.0)) < 1e-13
    lap = oracle.laplacian(P, (c * d).ravel())
    ddc = -1.0 + 1.5 * A1
    ddd = 0.6 - 3.6 * A2
    assert np.max(np.abs(lap - (ddc * d + c * ddd).ravel())) < 1e-10


def brute_free(n1, n2, z, gamma, eps, L=2.0):
    N = n1 * n2
    coef = -(L / n1) * (L / n2) / (4 * math.pi)
    u = np.zeros((3, N))
    for i in range(N):
        acc = [0.0, 0.0, 0.0]
        for j in range(N):
            r = [z[0][i] - z[0][j], z[1][i] - z[1][j], z[2][i] - z[2][j]]
            wgt = (r[0] ** 2 + r[1] ** 2 + r[2] ** 2 + eps * eps) ** -1.5
            g = gamma[:, j]
            acc[0] += wgt * (r[1] * g[2] - r[2] * g[1])
            acc[1] += wgt * (r[2] * g[0] - r[0] * g[2])
            acc[2] += wgt * (r[0] * g[1] - r[1] * g[0])
        u[:, i] = [coef * a for a in acc]
    return u


@pytest.mark.parametrize("n1,n2,seed", [(8, 8, 0), (9, 8, 1), (10, 12, 2)])
def test_free_br_matches_brute_force(n1, n2, seed):
    P = prob(n1, n2)
    z, w = rr.random_state(n1, n2, seed=seed, height=0.2)
    _, _, gam, _ = oracle.surface(P, z, w)
    assert relerr(oracle.br_velocity(P, z, w), brute_free(n1, n2, z, gam, P.eps)) < 1e-13


def test_free_rigid_translation():
    n = 16
    P = prob(n)
    z, w = rr.random_state(n, n, seed=3, height=0.1)
    u = oracle.br_velocity(P, z, w)
    zt = z + np.array([[0.731], [-1.37], [0.29]])
    assert relerr(oracle.br_velocity(P, zt, w), u) < 1e-13


def test_free_mirror_symmetry():
    """Reverse the axis-1 index, negate z1 and w1: u1 flips sign, u2 and u3
    follow the relabelling (summation order aside)."""
    n1, n2 = 14, 10
    P = prob(n1, n2)
    z, w = rr.random_state(n1, n2, seed=4, height=0.1)
    zt, wt = oracle.rhs(P, z, w)
    Z = z.reshape(3, n2, n1)[:, :, ::-1].copy(); W = w.reshape(2, n2, n1)[:, :, ::-1].copy()
    Z[0] = -Z[0]; W[0] = -W[0]
    mzt, mwt = oracle.rhs(P, Z.reshape(3, -1), W.reshape(2, -1))
    ref_z = zt.reshape(3, n2, n1)[:, :, ::-1].copy(); ref_z[0] = -ref_z[0]
    ref_w = wt.reshape(2, n2, n1)[:, :, ::-1].copy(); ref_w[0] = -ref_w[0]
    assert relerr(mzt.reshape(3, n2, n1), ref_z) < 1e-13
    assert relerr(mwt.reshape(2, n2, n1), ref_w) < 1e-13


def test_free_differs_from_periodic_at_the_edges_only_through_ghosts_and_images():
    """Far from the edges the stencils agree with the periodic ones; the BR
    sums differ (images), so only the tangents are compared."""
    n = 24
    z, _ = rr.single_mode(n, n, 0.05)
    tf1, tf2 = oracle.tangents(prob(n), z)
    tp1, tp2 = oracle.tangents(oracle.Problem(n, n, eps=1 / n), z)
    inner = np.zeros((n, n), bool); inner[2:-2, 2:-2] = True
    assert np.array_equal(tf1[:, inner.ravel()], tp1[:, inner.ravel()])
    assert not np.allclose(tf1[:, ~inner.ravel()], tp1[:, ~inner.ravel()], rtol=0, atol=1e-14)


def brute_free_cutoff(n1, n2, z, gamma, eps, rc, L=2.0):
    """Free-space sum over the sources strictly within rc of the target
    (3D distance, no images)."""
    N = n1 * n2
    coef = -(L / n1) * (L / n2) / (4 * math.pi)
    u = np.zeros((3, N))
    count = 0
    for i in range(N):
        acc = [0.0, 0.0, 0.0]
        for j in range(N):
            r = [z[0][i] - z[0][j], z[1][i] - z[1][j], z[2][i] - z[2][j]]
            dd = r[0] ** 2 + r[1] ** 2 + r[2] ** 2
            if not dd < rc * rc:
                continue
            count += 1
            wgt = (dd + eps * eps) ** -1.5
            g = gamma[:, j]
            acc[0] += wgt * (r[1] * g[2] - r[2] * g[1])
            acc[1] += wgt * (r[2] * g[0] - r[0] * g[2])
            acc[2] += wgt * (r[0] * g[1] - r[1] * g[0])
        u[:, i] = [coef * a for a in acc]
    return u, count


@pytest.mark.parametrize("n1,n2,rc,seed", [(8, 8, 0.3, 6), (10, 9, 0.75, 7), (9, 12, 1.3, 8)])
def test_free_cutoff_matches_brute_force(n1, n2, rc, seed):
    """rc up to 0.65 of the side: a periodic sheet would take the nearer
    image of a far-apart pair, a free one never does."""
    P = prob(n1, n2, cutoff=rc)
    z, w = rr.random_state(n1, n2, seed=seed, height=0.2)
    _, _, gam, _ = oracle.surface(P, z, w)
    ref, count = brute_free_cutoff(n1, n2, z, gam, P.eps, rc)
    assert 0 < count < (n1 * n2) ** 2
    assert relerr(oracle.br_velocity(P, z, w), ref) < 1e-13


def test_free_cutoff_beyond_the_diameter_is_the_exact_sum():
    """Once rc exceeds every pair distance the cutoff sum is the exact free
    sum: same terms, same order."""
    n = 12
    z, w = rr.random_state(n, n, seed=9, height=0.2)
    z[0] += 5.0                          # far outside the period cell: nothing wraps
    exact = oracle.br_velocity(prob(n), z, w)
    assert relerr(oracle.br_velocity(prob(n, cutoff=3.5), z, w), exact) < 1e-15


def test_free_cutoff_rhs_and_steps_run():
    n = 12
    P = prob(n, cutoff=0.6, dt=1e-3)
    z, _ = rr.single_mode(n, n, 0.05)
    w = rr.synthetic_vorticity(n, n, seed=10, sigma=0.02)
    z1, w1 = oracle.rk3(P, z, w, 2)
    assert np.all(np.isfinite(z1)) and np.all(np.isfinite(w1))
    assert not np.array_equal(w1, w)


def test_free_rejects_unsupported():
    z, w = rr.random_state(8, 8, seed=5)
    for kw in ({"images": 1}, {"model": 1}, {"cutoff": -0.1}):
        with pytest.raises(ValueError):
            oracle.br_velocity(prob(8, **kw), z, w)
