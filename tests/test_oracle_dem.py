"""Pins of the rigid-body run oracle against what the mathematics fixes: the bridge search against
brute force over all periodic images, the discrete two-body motion under a constant attraction
(closed form of the semi-implicit Euler update), the contact's coefficient of restitution
against the damped-oscillator formula, and conservation of total momentum."""
import math

import numpy as np

from oracle import dem_oracle as D


def test_bridge_search_against_all_images():
    rng = np.random.default_rng(1)
    L, n, gmax = 40.0, 40, 3.0
    R = rng.uniform(2.0, 4.0, n)
    x = rng.uniform(0.0, L, (n, 3))
    ij, gaps, units = D.bridges(x, R, L, gmax)
    expect = {}
    shifts = [np.array(s) * L for s in np.ndindex(3, 3, 3)]
    for i in range(n):
        for j in range(i + 1, n):
            g = min(float(np.linalg.norm(x[j] + s - L - x[i])) for s in shifts) - R[i] - R[j]
            if g < gmax:
                expect[(i, j)] = g
    assert [tuple(p) for p in ij] == sorted(expect)
    for (i, j), g, e in zip(ij, gaps, units):
        assert abs(g - expect[(i, j)]) < 1e-12
        assert abs(np.linalg.norm(e) - 1.0) < 1e-14


def test_constant_attraction_closed_form():
    # two equal spheres, constant attraction F: relative gap after n steps of the semi-implicit
    # update is g0 - 2 (F / m) dt^2 n (n + 1) / 2 (both move towards each other)
    L, R, F, dt, rho = 100.0, 5.0, 0.3, 0.7, 2.0
    x = np.array([[40.0, 50.0, 50.0], [51.0, 50.0, 50.0]])
    v = np.zeros_like(x)
    Rs = np.array([R, R])
    m = rho * 4.0 / 3.0 * math.pi * R ** 3
    g0 = 1.0
    for n in range(1, 11):
        x, v, _ = D.step(x, v, Rs, L, dt, rho, 0.0, 0.0, 5.0, lambda ij, g: np.full(len(ij), F))
        g = x[1, 0] - x[0, 0] - 2 * R
        assert abs(g - (g0 - 2 * (F / m) * dt * dt * n * (n + 1) / 2)) < 1e-12


def test_contact_restitution():
    # head-on collision, spring-dashpot only: e = exp(-zeta pi / sqrt(1 - zeta^2)),
    # zeta = gamma / (2 sqrt(k m_eff)); the discrete update converges to it as dt -> 0
    L, R, rho, k, gam = 200.0, 4.0, 1.0, 2.0, 3.0
    m = rho * 4.0 / 3.0 * math.pi * R ** 3
    meff = m / 2
    zeta = gam / (2 * math.sqrt(k * meff))
    e_exact = math.exp(-zeta * math.pi / math.sqrt(1 - zeta ** 2))
    dt = 2 * math.pi / math.sqrt(k / meff) / 2000
    x = np.array([[90.0, 100.0, 100.0], [90.0 + 2 * R + 0.5, 100.0, 100.0]])
    u = 0.05
    v = np.array([[u, 0, 0], [-u, 0, 0]], dtype=float)
    Rs = np.array([R, R])
    for _ in range(20000):
        x, v, _ = D.step(x, v, Rs, L, dt, rho, k, gam, 1e-9, lambda ij, g: np.zeros(len(ij)))
        if v[1, 0] - v[0, 0] > 0 and x[1, 0] - x[0, 0] > 2 * R:
            break
    else:
        raise AssertionError("the spheres did not separate")
    e = (v[1, 0] - v[0, 0]) / (2 * u)
    assert abs(e - e_exact) < 2e-3


def test_momentum_conserved():
    rng = np.random.default_rng(4)
    L, n = 30.0, 30
    R = rng.uniform(1.5, 2.5, n)
    x = rng.uniform(0, L, (n, 3))
    v = rng.normal(0, 0.01, (n, 3))
    m = 3.0 * 4.0 / 3.0 * math.pi * R ** 3
    p0 = (m[:, None] * v).sum(0)
    for _ in range(50):
        x, v, _ = D.step(x, v, R, L, 0.5, 3.0, 5.0, 1.0, 2.0, lambda ij, g: 0.1 * np.cos(g))
    assert np.abs((m[:, None] * v).sum(0) - p0).max() < 1e-12 * max(1.0, np.abs(m[:, None] * v).sum())


def test_features_special_cases():
    f, rs = D.features([3.0], [3.0], [-0.5], 0.4, 0.2, 0.25)
    # equal radii: R* = R, ratio 1, V_L = 0.25 * 2 * (4/3) pi R^3, gap clamped at gap_min
    assert rs[0] == 3.0 and f[0, 1] == 1.0
    assert abs(f[0, 0] - 0.25 / 3.0) < 1e-15
    assert abs(f[0, 2] - 0.25 * 2 * 4 / 3 * math.pi) < 1e-13
    assert f[0, 3] == 0.4
