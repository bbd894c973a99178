"""Seeded synthetic inputs for the rocket-rig interface problem.

The paper's driver initialises a Rayleigh-Taylor interface between two fluids
with configurable initial conditions (sec. 4, rocket rig driver; periodic
multi-mode and single-mode test cases).  This module only draws those inputs:
it holds none of the solver's arithmetic and is shared by the CPU oracle's
tests and the GPU path alike.

Conventions
-----------
* Mesh of n1 x n2 points on the periodic parameter square [-1, 1)^2
  (period 2 on each axis), spacing h_a = 2 / n_a, node i at -1 + i h.
* Position planes z[3, N] with z = (alpha_1, alpha_2, h0(alpha)); vorticity
  planes w[2, N]; point index p = i2 * n1 + i1.
* Random numbers: ``numpy.random.default_rng(seed)`` (PCG64).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

PERIOD = 2.0


def grid(n1: int, n2: int):
    """Parameter coordinates (alpha_1, alpha_2) as (n2, n1) arrays."""
    a1 = -1.0 + np.arange(n1, dtype=np.float64) * (PERIOD / n1)
    a2 = -1.0 + np.arange(n2, dtype=np.float64) * (PERIOD / n2)
    A1, A2 = np.meshgrid(a1, a2, indexing="xy")
    return A1, A2


def flat_state(n1: int, n2: int):
    """Flat interface at rest: z = (alpha_1, alpha_2, 0), w = 0."""
    A1, A2 = grid(n1, n2)
    z = np.stack([A1, A2, np.zeros_like(A1)]).reshape(3, n1 * n2)
    w = np.zeros((2, n1 * n2))
    return z, w


def single_mode(n1: int, n2: int, amplitude: float, noise: float = 0.0, seed: int = 0):
    """h0 = amplitude cos(pi x) cos(pi y) (+ i.i.d. U(-noise, noise) per point)."""
    z, w = flat_state(n1, n2)
    A1, A2 = grid(n1, n2)
    h = amplitude * np.cos(math.pi * A1) * np.cos(math.pi * A2)
    if noise > 0.0:
        rng = np.random.default_rng(seed)
        h = h + rng.uniform(-noise, noise, size=h.shape)
    z[2] = h.ravel()
    return z, w


def multi_mode(n1: int, n2: int, modes: int, seed: int, sigma: float = 0.01,
               noise: float = 1e-4):
    """h0 = sum_{m=1..M} a_m cos(m pi x + phi_m) cos(m pi y + psi_m) + noise.

    a_m ~ N(0, sigma^2), phi_m, psi_m ~ U[0, 2 pi), drawn in the order
    (a_m, phi_m, psi_m) for m = 1..M; then i.i.d. U(-noise, noise) per point
    in point order.
    """
    z, w = flat_state(n1, n2)
    A1, A2 = grid(n1, n2)
    rng = np.random.default_rng(seed)
    h = np.zeros_like(A1)
    for m in range(1, modes + 1):
        a = rng.normal(0.0, sigma)
        phi = rng.uniform(0.0, 2.0 * math.pi)
        psi = rng.uniform(0.0, 2.0 * math.pi)
        h = h + a * np.cos(m * math.pi * A1 + phi) * np.cos(m * math.pi * A2 + psi)
    if noise > 0.0:
        h = h + rng.uniform(-noise, noise, size=h.shape)
    z[2] = h.ravel()
    return z, w


def synthetic_vorticity(n1: int, n2: int, seed: int, modes: int = 8, sigma: float = 0.01):
    """w = grad(mu) (analytic) for mu = sum_m b_m cos(m pi x + p_m) cos(m pi y + s_m).

    Used where a non-zero vorticity is needed for a BR-only evaluation (the
    physical initial vorticity is zero).  b_m ~ N(0, sigma^2), phases
    U[0, 2 pi), drawn in the order (b_m, p_m, s_m); the stream is
    default_rng(seed + 1000) so it is independent of the interface draw.
    """
    A1, A2 = grid(n1, n2)
    rng = np.random.default_rng(seed + 1000)
    w1 = np.zeros_like(A1)
    w2 = np.zeros_like(A1)
    for m in range(1, modes + 1):
        b = rng.normal(0.0, sigma)
        p = rng.uniform(0.0, 2.0 * math.pi)
        s = rng.uniform(0.0, 2.0 * math.pi)
        k = m * math.pi
        w1 = w1 - b * k * np.sin(k * A1 + p) * np.cos(k * A2 + s)
        w2 = w2 - b * k * np.cos(k * A1 + p) * np.sin(k * A2 + s)
    return np.stack([w1, w2]).reshape(2, n1 * n2)


def random_state(n1: int, n2: int, seed: int, height: float = 0.05, modes: int = 4):
    """A smooth non-flat interface with non-zero vorticity, for parity tests."""
    z, _ = multi_mode(n1, n2, modes, seed, sigma=height, noise=0.0)
    w = synthetic_vorticity(n1, n2, seed, modes=modes, sigma=0.05)
    return z, w


def sample_targets(n: int, count: int, seed: int) -> np.ndarray:
    """Distinct seeded point indices (sorted)."""
    rng = np.random.default_rng(seed + 2000)
    count = min(count, n)
    return np.sort(rng.choice(n, size=count, replace=False)).astype(np.int64)


# --------------------------------------------------------------------------
# Named workloads (sizes and draws only)
# --------------------------------------------------------------------------

@dataclass
class Workload:
    name: str
    n1: int
    n2: int
    atwood: float
    gravity: float
    dt: float
    steps: int
    eps_over_h: float
    seed: int
    precision: str            # "fp64" or "fp32_pairs"
    kind: str                 # "single_mode_noise" | "multi_mode"
    modes: int = 0
    amplitude: float = 0.0
    noise: float = 0.0
    extra: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.n1 * self.n2

    @property
    def eps(self) -> float:
        return self.eps_over_h * (PERIOD / self.n1)

    def state(self):
        if self.kind == "single_mode_noise":
            return single_mode(self.n1, self.n2, self.amplitude, self.noise, self.seed)
        if self.kind == "multi_mode":
            return multi_mode(self.n1, self.n2, self.modes, self.seed, noise=self.noise)
        raise ValueError(self.kind)

    def pairs_per_step(self) -> int:
        return 3 * self.n * self.n


WORKLOADS = {
    # 64 x 64 single mode + 1e-4 noise, FP64, 10 steps (oracle finishes in seconds)
    "periodic64_single_fp64": Workload(
        "periodic64_single_fp64", 64, 64, atwood=0.5, gravity=1.0, dt=1e-3, steps=10,
        eps_over_h=0.5, seed=0, precision="fp64", kind="single_mode_noise",
        amplitude=0.05, noise=1e-4),
    # 256 x 256, 8 seeded modes + noise, FP64, 50 steps
    "periodic256_multimode8_fp64": Workload(
        "periodic256_multimode8_fp64", 256, 256, atwood=0.5, gravity=1.0, dt=1e-3, steps=50,
        eps_over_h=0.5, seed=1, precision="fp64", kind="multi_mode", modes=8, noise=1e-4),
    # 1024 x 1024, 16 seeded modes + noise, FP32 pair interactions, 5 steps
    "periodic1024_multimode16_fp32": Workload(
        "periodic1024_multimode16_fp32", 1024, 1024, atwood=0.9, gravity=1.0, dt=1e-3, steps=5,
        eps_over_h=0.5, seed=2, precision="fp32_pairs", kind="multi_mode", modes=16, noise=1e-4),
}


# --------------------------------------------------------------------------
# Ensembles and request streams (sizes and draws only)
# --------------------------------------------------------------------------

ENSEMBLE_SIDES = (32, 48, 64, 96, 128, 192, 256)


@dataclass
class Member:
    """One simulation of an ensemble or a request stream."""
    n: int                    # mesh side (n x n)
    atwood: float
    amplitude: float          # single-mode amplitude a cos(pi x) cos(pi y)
    steps: int = 0
    arrival: float = 0.0      # seconds after the stream starts (requests only)

    @property
    def eps(self) -> float:
        return 0.5 * PERIOD / self.n

    def state(self):
        return single_mode(self.n, self.n, self.amplitude)


def ensemble(count: int = 64, seed: int = 3):
    """Uneven ensemble: per member, in this order, side ~ U{32,...,256},
    A ~ U[0.1, 0.9], amplitude ~ U[0.01, 0.1]; single mode, no noise."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        n = int(rng.choice(ENSEMBLE_SIDES))
        a = float(rng.uniform(0.1, 0.9))
        amp = float(rng.uniform(0.01, 0.1))
        out.append(Member(n, a, amp))
    return out


def request_stream(count: int = 200, rate: float = 1.0, seed: int = 4,
                   side_min: int = 64, side_max: int = 512, steps_min: int = 100,
                   steps_max: int = 1000):
    """Poisson arrivals at `rate` per second.  Per request, in this order:
    inter-arrival ~ Exp(rate), side = exp(U(ln side_min, ln side_max)) rounded
    to a multiple of 8, A ~ U[0.1, 0.9], steps ~ U{steps_min..steps_max},
    amplitude ~ U[0.01, 0.1]."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for _ in range(count):
        t += float(rng.exponential(1.0 / rate))
        side = float(np.exp(rng.uniform(math.log(side_min), math.log(side_max))))
        n = int(max(8, 8 * round(side / 8)))
        a = float(rng.uniform(0.1, 0.9))
        steps = int(rng.integers(steps_min, steps_max + 1))
        amp = float(rng.uniform(0.01, 0.1))
        out.append(Member(n, a, amp, steps=steps, arrival=t))
    return out
