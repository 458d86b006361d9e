"""Plain FP64 NumPy reference of the many-sphere rigid-body run with pairwise bridge forces
(test infrastructure).

TEST INFRASTRUCTURE ONLY: used by the test suite to check the GPU run; the product path never
imports it.

Model (the definitions the GPU run implements):
* periodic cube of edge L, minimum-image separation d_ij = x_j - x_i, r = |d_ij|, unit e = d / r;
* surface gap g = r - (R_i + R_j); a bridge joins i and j iff g < gap_max (Sec. 2.2 fixes a
  bridge by the gap, the radii, the liquid volume and the contact angle);
* bridge features (max(g, gap_min) / R*, min(R) / max(R), V_L / R*^3, theta) with
  R* = 2 R_i R_j / (R_i + R_j) and V_L = c / (1 - c) (4/3) pi (R_i^3 + R_j^3);
* bridge force on i: F_b e, F_b = f R*, f the de-normalised network output (attractive);
* contact (g < 0): k_n g e + gamma_n ((v_j - v_i) . e) e on i (spring and dashpot);
* semi-implicit Euler of the rigid bodies (Sec. 3.3): v += F / m dt, then x += v dt, wrapped into
  [0, L); m = density (4/3) pi R^3.
Pins: tests/test_oracle_dem.py (brute-force bridge search, two-body closed forms of the discrete
update, contact restitution, momentum conservation).
"""
from __future__ import annotations

import math

import numpy as np


def min_image(d, L):
    return d - L * np.floor(d / L + 0.5)


def bridges(x, R, L, gap_max):
    """Bridged pairs (i < j) in (i, j) order, their gaps and unit vectors e_ij (from i to j)."""
    n = len(R)
    ij, gaps, units = [], [], []
    for i in range(n):
        d = min_image(x[i + 1:] - x[i], L)
        r = np.sqrt((d * d).sum(axis=1))
        g = r - (R[i] + R[i + 1:])
        for k in np.nonzero(g < gap_max)[0]:
            ij.append((i, i + 1 + k))
            gaps.append(g[k])
            units.append(d[k] / r[k])
    return (np.array(ij, dtype=np.int64).reshape(-1, 2), np.array(gaps, dtype=np.float64),
            np.array(units, dtype=np.float64).reshape(-1, 3))


def features(Ri, Rj, gap, theta, c, gap_min):
    Ri, Rj, gap = (np.asarray(a, dtype=np.float64) for a in (Ri, Rj, gap))
    rs = 2.0 * Ri * Rj / (Ri + Rj)
    vl = c / (1.0 - c) * (4.0 / 3.0) * math.pi * (Ri ** 3 + Rj ** 3)
    f = np.stack([np.maximum(gap, gap_min) / rs, np.minimum(Ri, Rj) / np.maximum(Ri, Rj), vl / rs ** 3,
                  np.full_like(rs, theta)], axis=1)
    return f, rs


def forces(x, v, R, L, ij, units, gaps, bridge_force, k_n, gamma_n):
    """Per-sphere force from the bridge forces F_b of the pairs ij and the contact law."""
    F = np.zeros_like(x)
    for (i, j), e, g, fb in zip(ij, units, gaps, bridge_force):
        fn = fb
        if g < 0.0:
            fn += k_n * g + gamma_n * float(np.dot(v[j] - v[i], e))
        F[i] += fn * e
        F[j] -= fn * e
    return F


def integrate(x, v, F, R, density, dt, L):
    m = density * (4.0 / 3.0) * math.pi * R ** 3
    v = v + F / m[:, None] * dt
    x = x + v * dt
    x = x - L * np.floor(x / L)
    x[x >= L] -= L
    return x, v


def step(x, v, R, L, dt, density, k_n, gamma_n, gap_max, bridge_force_fn):
    """One step; bridge_force_fn(ij, gaps) returns F_b for every bridge."""
    ij, gaps, units = bridges(x, R, L, gap_max)
    fb = bridge_force_fn(ij, gaps) if len(ij) else np.zeros(0)
    F = forces(x, v, R, L, ij, units, gaps, fb, k_n, gamma_n)
    x, v = integrate(x, v, F, R, density, dt, L)
    return x, v, F
