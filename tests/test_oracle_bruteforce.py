"""High-precision brute force on tiny meshes (40 significant digits).

This checks the oracle's FP64 arithmetic (compensated sums, the order of
operations, the seam bookkeeping on tiny meshes) rather than its formulas:
the formulas are pinned by closed forms and symmetries in
test_oracle_pins.py.  The brute force follows the same definitions directly:
5-point tangents with the periodic coordinate correction, source strength
w1 T2 - w2 T1, index-based minimum image with split ties, and
u = -(h1 h2 / 4 pi) sum c (r x gamma) / (|r|^2 + eps^2)^(3/2).
"""
import numpy as np
import pytest

mpmath = pytest.importorskip("mpmath")

import oracle
import rocket_rig as rr

mp = mpmath.mp


def _brute(n1, n2, z, w, eps):
    mp.dps = 40
    L = mp.mpf(2)
    N = n1 * n2
    Z = [[mp.mpf(float(v)) for v in z[c]] for c in range(3)]
    W = [[mp.mpf(float(v)) for v in w[c]] for c in range(2)]
    h1, h2 = L / n1, L / n2

    def zat(c, i1, i2):
        w1, j1 = divmod(i1, n1)
        w2, j2 = divmod(i2, n2)
        v = Z[c][j2 * n1 + j1]
        if c == 0:
            v += w1 * L
        if c == 1:
            v += w2 * L
        return v

    def d(fm2, fm1, fp1, fp2, h):
        return (8 * (fp1 - fm1) - (fp2 - fm2)) / (12 * h)

    G = [[None] * N for _ in range(3)]
    for i2 in range(n2):
        for i1 in range(n1):
            p = i2 * n1 + i1
            T1 = [d(zat(c, i1 - 2, i2), zat(c, i1 - 1, i2), zat(c, i1 + 1, i2), zat(c, i1 + 2, i2), h1)
                  for c in range(3)]
            T2 = [d(zat(c, i1, i2 - 2), zat(c, i1, i2 - 1), zat(c, i1, i2 + 1), zat(c, i1, i2 + 2), h2)
                  for c in range(3)]
            for c in range(3):
                G[c][p] = W[0][p] * T2[c] - W[1][p] * T1[c]

    def images(i, j, n):
        dd = (j - i) % n
        if 2 * dd < n:
            return [((i + dd - j) // n, mp.mpf(1))]
        if 2 * dd > n:
            return [((i + dd - n - j) // n, mp.mpf(1))]
        half = mp.mpf(1) / 2
        return [((i + dd - j) // n, half), ((i + dd - n - j) // n, half)]

    e2 = mp.mpf(float(eps)) ** 2
    coef = -(h1 * h2) / (4 * mp.pi)
    u = np.zeros((3, N))
    for i2 in range(n2):
        for i1 in range(n1):
            pi_ = i2 * n1 + i1
            acc = [mp.mpf(0)] * 3
            for j2 in range(n2):
                for j1 in range(n1):
                    pj = j2 * n1 + j1
                    for s2, c2 in images(i2, j2, n2):
                        for s1, c1 in images(i1, j1, n1):
                            r = [Z[0][pi_] - Z[0][pj] - s1 * L, Z[1][pi_] - Z[1][pj] - s2 * L,
                                 Z[2][pi_] - Z[2][pj]]
                            g = [G[0][pj], G[1][pj], G[2][pj]]
                            f = c1 * c2 / (r[0] ** 2 + r[1] ** 2 + r[2] ** 2 + e2) ** mp.mpf(1.5)
                            acc[0] += f * (r[1] * g[2] - r[2] * g[1])
                            acc[1] += f * (r[2] * g[0] - r[0] * g[2])
                            acc[2] += f * (r[0] * g[1] - r[1] * g[0])
            for c in range(3):
                u[c, pi_] = float(coef * acc[c])
    return u


@pytest.mark.slow
@pytest.mark.parametrize("n1,n2,seed", [(8, 8, 0), (8, 12, 1), (10, 10, 2), (9, 7, 3)])
def test_oracle_matches_bruteforce(n1, n2, seed):
    z, w = rr.random_state(n1, n2, seed=seed, height=0.15)
    eps = 0.5 * 2.0 / n1
    u_ref = _brute(n1, n2, z, w, eps)
    u = oracle.br_velocity(oracle.Problem(n1, n2, eps=eps), z, w)
    err = np.max(np.abs(u - u_ref)) / np.max(np.abs(u_ref))
    assert err < 1e-15
