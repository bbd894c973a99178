"""Pins of the oracle's low-order velocity (CPU only).

The low-order model replaces the BR sum by its flat-sheet approximation
u = 1/2 (R1 w1 + R2 w2) n^, R_a the Riesz transform (symbol i k_a / |k|)
over the periodic mesh.  Checked against:
  * the flat sheet carrying a plane wave, where the symbol gives exactly
    u3 = -|k|/2 mu;
  * numpy's FFT (an independent library) on random fields and meshes;
  * the unpaired Nyquist mode, which gives zero (the rule that zeroes its
    symbol does not change the real part: i k_a times a real Nyquist
    coefficient is imaginary and drops out);
  * the linear Rayleigh-Taylor growth rate sigma^2 = A g (k . k~) / |k|
    (k~ the 5-point modified wavenumbers of D V), through RK3;
  * the sign symmetry in w.
"""
import math

import numpy as np
import pytest

import oracle
import rocket_rig as rr


def prob(n1, n2=None, **kw):
    n2 = n1 if n2 is None else n2
    kw.setdefault("eps", 0.5 * 2.0 / n1)
    return oracle.Problem(n1, n2, model=1, **kw)


def relerr(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / np.max(np.abs(b)))


def plane_wave(n1, n2, k1, k2, L1=2.0, L2=2.0):
    a1 = -0.5 * L1 + np.arange(n1) * (L1 / n1)
    a2 = -0.5 * L2 + np.arange(n2) * (L2 / n2)
    A1, A2 = np.meshgrid(a1, a2)
    mu = np.cos(k1 * A1 + k2 * A2).ravel()
    s = np.sin(k1 * A1 + k2 * A2).ravel()
    z = np.stack([A1.ravel(), A2.ravel(), np.zeros(n1 * n2)])
    return z, np.stack([-k1 * s, -k2 * s]), mu


@pytest.mark.parametrize("n1,n2,m1,m2,L1,L2", [
    (16, 16, 1, 0, 2.0, 2.0), (16, 16, 1, 2, 2.0, 2.0), (12, 20, 3, -2, 2.0, 2.0),
    (9, 15, 2, 4, 2.0, 2.0), (16, 8, 1, 1, 3.0, 1.5),
])
def test_low_order_flat_sheet_symbol(n1, n2, m1, m2, L1, L2):
    k1, k2 = 2 * math.pi * m1 / L1, 2 * math.pi * m2 / L2
    z, w, mu = plane_wave(n1, n2, k1, k2, L1, L2)
    u = oracle.br_velocity(prob(n1, n2, period1=L1, period2=L2), z, w)
    assert np.all(u[:2] == 0.0)
    assert np.max(np.abs(u[2] + 0.5 * math.hypot(k1, k2) * mu)) < 1e-13 * math.hypot(k1, k2)


def numpy_low_order(P, z, w):
    """The same definition through numpy's FFT."""
    n1, n2 = P.n1, P.n2
    W1 = np.fft.fft2(w[0].reshape(n2, n1))
    W2 = np.fft.fft2(w[1].reshape(n2, n1))
    m1 = np.fft.fftfreq(n1, 1.0 / n1)
    m2 = np.fft.fftfreq(n2, 1.0 / n2)
    M1, M2 = np.meshgrid(m1, m2)
    K1 = 2 * np.pi * M1 / P.period1
    K2 = 2 * np.pi * M2 / P.period2
    KK = np.hypot(K1, K2)
    with np.errstate(invalid="ignore", divide="ignore"):
        c1 = np.where(KK > 0, K1 / KK, 0.0)
        c2 = np.where(KK > 0, K2 / KK, 0.0)
    if n1 % 2 == 0:
        c1[:, n1 // 2] = 0.0
    if n2 % 2 == 0:
        c2[n2 // 2, :] = 0.0
    S = np.real(np.fft.ifft2(0.5j * (c1 * W1 + c2 * W2))).ravel()
    t1, t2 = oracle.tangents(P, z)
    nrm = np.cross(t1.T, t2.T).T
    nrm = nrm / np.linalg.norm(nrm, axis=0)
    return S * nrm


@pytest.mark.parametrize("n1,n2,L1,L2,seed", [(8, 8, 2.0, 2.0, 0), (12, 10, 2.0, 2.0, 1),
                                              (9, 7, 2.0, 2.0, 2), (16, 12, 3.0, 1.5, 3)])
def test_low_order_matches_numpy_fft(n1, n2, L1, L2, seed):
    P = prob(n1, n2, period1=L1, period2=L2)
    z, w = rr.random_state(n1, n2, seed=seed, height=0.1)
    z[0] *= L1 / 2.0
    z[1] *= L2 / 2.0
    u = oracle.br_velocity(P, z, w)
    assert relerr(u, numpy_low_order(P, z, w)) < 1e-13


def test_low_order_nyquist_mode_is_zero():
    n1, n2 = 16, 12
    z, _ = rr.flat_state(n1, n2)
    j1 = np.arange(n1)
    w = np.zeros((2, n1 * n2))
    w[0] = np.tile((-1.0) ** j1, n2)
    w[1] = np.repeat((-1.0) ** np.arange(n2), n1)
    u = oracle.br_velocity(prob(n1, n2), z, w)
    assert np.max(np.abs(u)) < 1e-14


def test_low_order_linear_growth_through_rk3():
    """Tiny single mode, w0 = 0: the amplitude follows R(dt M)^n with
    M = [[0, 1], [sigma^2, 0]], sigma^2 = A g (k . k~) / |k|."""
    n, A, g, dt, steps = 32, 0.5, 1.0, 5e-3, 40
    m1, m2 = 1, 2
    h = 2.0 / n
    k = np.array([math.pi * m1, math.pi * m2])
    kt = (8 * np.sin(k * h) - np.sin(2 * k * h)) / (6 * h)
    sig2 = A * g * float(k @ kt) / float(np.linalg.norm(k))
    amp = 1e-7
    A1, A2 = rr.grid(n, n)
    mode = np.cos(k[0] * A1 + k[1] * A2).ravel()
    z, w = rr.flat_state(n, n)
    z[2] = amp * mode
    P = prob(n, atwood=A, gravity=g, dt=dt)
    zn, _ = oracle.rk3(P, z, w, steps)
    a_n = float(zn[2] @ mode / (mode @ mode))
    M = np.array([[0.0, 1.0], [sig2, 0.0]]) * dt
    R = np.eye(2) + M + M @ M / 2 + M @ M @ M / 6
    y = np.linalg.matrix_power(R, steps) @ np.array([amp, 0.0])
    assert abs(a_n / y[0] - 1) < 1e-5


def test_low_order_sign_symmetry_bitwise():
    n = 12
    z, w = rr.random_state(n, n, seed=4, height=0.1)
    P = prob(n)
    u = oracle.br_velocity(P, z, w)
    assert np.array_equal(oracle.br_velocity(P, z, -w), -u)


def test_low_order_rejects_sampling_and_cutoff():
    z, w = rr.random_state(8, 8, seed=5)
    with pytest.raises(ValueError):
        oracle.br_velocity(prob(8), z, w, targets=[0, 1])
    with pytest.raises(ValueError):
        oracle.br_velocity(prob(8, cutoff=0.3), z, w)


@pytest.mark.parametrize("n1,n2,L1,L2", [(16, 16, 2.0, 2.0), (32, 8, 2.0, 2.0), (8, 32, 3.0, 1.5)])
def test_numpy_fft_reference_matches_oracle(n1, n2, L1, L2):
    """The numpy-FFT evaluation the large GPU tests compare with agrees with
    the oracle's direct DFT sums."""
    from zm_testutil import fft_reference
    z, w = rr.random_state(n1, n2, seed=n1 + n2, height=0.1)
    z[0] *= L1 / 2.0
    z[1] *= L2 / 2.0
    P = oracle.Problem(n1, n2, eps=1.0 / n1, period1=L1, period2=L2, model=1)
    u = oracle.br_velocity(P, z, w)
    ref = fft_reference(n1, n2, z, w, L1, L2)
    assert np.max(np.abs(ref - u)) < 1e-13 * np.max(np.abs(u))
