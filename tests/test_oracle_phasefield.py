"""Pins of the oracle's phase-field update (Sec. 3.1.1 advection with directional splitting and an
MC limiter; Sec. 3.3 multi-phase-field kinetics).

Expectations: exact integer shift at Courant number 1, exact conservation and bounds of the
conservative split scheme, exact per-step amplification of Fourier modes under the explicit
kinetics (derived below from the equation of Sec. 3.3 and the 7-point Laplacian's symbol), a
discrete-eigenfunction profile that the kinetics leaves unchanged, and the sum constraint."""
import math

import numpy as np
import pytest

from oracle_helpers import body, params
from pflbm_inputs import sphere_phi


def _pf_only(oracle_mod, shape, phis, bodies, **over):
    """Phase fields on an empty fluid (rho = 0), so the fluid exerts no force."""
    over.setdefault("G", 0.0)
    p = params(shape, len(bodies), **over)
    return oracle_mod.Oracle(p, bodies, np.zeros(shape), np.asarray(phis))


@pytest.mark.parametrize("v,axis,sign", [((1, 0, 0), 3, 1), ((0, -1, 0), 2, -1), ((0, 0, 1), 1, 1)])
def test_advection_courant_one_is_exact_shift(oracle_mod, v, axis, sign):
    """At |u| = 1 the MC-limited flux is the upwind value and each step shifts by one cell."""
    shape = (9, 10, 11)
    phi = sphere_phi(shape, (5.2, 4.8, 4.1), 2.7, 3.0)[None]
    o = _pf_only(oracle_mod, shape, phi, [body(v=v, fixed=1)], kinetics=0, motion=0)
    o.step(4)
    assert np.array_equal(o.phi(), np.roll(phi, 4 * sign, axis=axis))


def test_advection_conserves_and_bounds(oracle_mod):
    """Conservative split fluxes with a rigid (divergence-free) velocity: sum phi is conserved to
    round-off; each 1-D MC sweep is TVD for |u| <= 1, so phi stays in [0, 1]; the centroid moves
    with the body velocity."""
    shape = (28, 28, 34)  # the support stays clear of the periodic wrap for 20 steps
    phi = sphere_phi(shape, (10.0, 15.0, 11.2), 4.0, 3.0)[None]
    V = (0.37, -0.21, 0.13)
    o = _pf_only(oracle_mod, shape, phi, [body(v=V, w=(0.0, 0.0, 0.004), fixed=0)], kinetics=0, motion=1)
    s0 = phi.sum()
    o.step(20)
    p = o.phi()
    assert abs(p.sum() - s0) < 1e-12 * s0
    assert p.min() >= 0.0 and p.max() <= 1.0
    z, y, x = np.meshgrid(*(np.arange(n, dtype=float) for n in shape), indexing="ij")

    def centroid(f):
        return np.array([(f * x).sum(), (f * y).sum(), (f * z).sum()]) / f.sum()

    c0, c1 = centroid(phi[0]), centroid(p[0])
    assert np.allclose(c1 - c0, 20 * np.array(V), atol=0.05)


def test_kinetics_two_phase_fourier_mode(oracle_mod):
    """Two phases (fluid 0, solid 1), phi_1 = 1/2 + e cos(kx), both active everywhere (N = 2).
    With I_a = lap phi_a + mu phi_a, mu = pi^2/eta^2 and the 7-point Laplacian's symbol
    -lam_k, lam_k = 2 - 2 cos k:  I_1 - I_0 = 2 e cos(kx)(mu - lam_k), so the update
    phi_1 += (M/2) sigma (I_1 - I_0) multiplies e by 1 + M sigma (mu - lam_k) exactly per step
    (the volume term vanishes: the mean is unchanged)."""
    P, eps, M, sig, eta = 12, 0.1, 0.02, 1.3, 5.0
    shape = (1, 1, P)
    x = np.arange(P)
    k = 2 * math.pi / P
    phi = (0.5 + eps * np.cos(k * x)).reshape((1,) + shape)
    sigma = np.array([[0.0, sig], [sig, 0.0]])
    o = _pf_only(oracle_mod, shape, phi, [body(fixed=1)], kinetics=1, motion=0, mobility=M, eta=eta, sigma=sigma)
    n = 30
    o.step(n)
    mu, lam = math.pi ** 2 / eta ** 2, 2 - 2 * math.cos(k)
    want = 0.5 + eps * (1 + M * sig * (mu - lam)) ** n * np.cos(k * x)
    assert np.max(np.abs(o.phi()[0, 0, 0] - want)) < 1e-14


def test_kinetics_three_phase_fourier_mode(oracle_mod):
    """Three phases (fluid 0, solids 1, 2), phi_1 = a + d, phi_2 = a - d, phi_0 = c, d = e cos(kx),
    sigma_01 = sigma_02 = s, sigma_12 = g.  Summing the pair terms of Sec. 3.3 over beta in {0, 2}
    for alpha = 1 gives (M/3)[(s + g) I_1 + (s - 2g) I_2 - s I_0]; its mode part is
    M g (mu - lam_k) d, and its mean part vanishes for c = (2s - g) a / s.  The third-phase term
    (sigma_bg - sigma_ag) I_g enters with that sign; the opposite sign would give
    (2s + g)(mu - lam_k) d / 3 instead."""
    P, eps, M, s, g, eta = 10, 0.05, 0.03, 1.0, 0.5, 4.0
    a = 2.0 / 7.0
    c = (2 * s - g) * a / s
    assert abs(2 * a + c - 1.0) < 1e-15
    shape = (1, 1, P)
    x = np.arange(P)
    k = 2 * math.pi / P
    d = eps * np.cos(k * x)
    phi = np.stack([(a + d).reshape(shape), (a - d).reshape(shape)])
    sigma = np.array([[0.0, s, s], [s, 0.0, g], [s, g, 0.0]])
    o = _pf_only(oracle_mod, shape, phi, [body(fixed=1), body(fixed=1)], kinetics=1, motion=0,
                 mobility=M, eta=eta, sigma=sigma, repulsion=0)
    n = 20
    o.step(n)
    mu, lam = math.pi ** 2 / eta ** 2, 2 - 2 * math.cos(k)
    amp = (1 + M * g * (mu - lam)) ** n
    p = o.phi()
    assert np.max(np.abs(p[0, 0, 0] - (a + amp * d))) < 1e-14
    assert np.max(np.abs(p[1, 0, 0] - (a - amp * d))) < 1e-14


def test_kinetics_discrete_sine_profile_is_stationary(oracle_mod):
    """phi_1 = (1 + sin(k x + 1/4 k))/2 with k = 2 pi/P and eta chosen so that
    pi^2/eta^2 = lam_k: then I_1 - I_0 = 0 at every node and the profile does not move."""
    P = 10
    k = 2 * math.pi / P
    eta = math.pi / math.sqrt(2 - 2 * math.cos(k))
    shape = (1, 1, P)
    x = np.arange(P)
    phi = (0.5 * (1 + np.sin(k * (x + 0.25)))).reshape((1,) + shape)
    o = _pf_only(oracle_mod, shape, phi, [body(fixed=1)], kinetics=1, motion=0, mobility=0.05, eta=eta)
    o.step(50)
    assert np.max(np.abs(o.phi() - phi)) < 1e-13


def test_kinetics_keeps_sum_constraint_and_bounds(oracle_mod):
    """Three touching diffuse spheres under kinetics with a large mobility: every solid phase in
    [0, 1], the solid sum never above 1 (fluid fraction >= 0), and the update is antisymmetric in
    each pair, so away from the clip the phases exchange volume without creating any."""
    shape = (16, 16, 16)
    phis = np.stack([sphere_phi(shape, c, 3.5, 4.0) for c in ((5.0, 8.0, 8.0), (11.0, 8.0, 8.0), (8.0, 13.0, 8.0))])
    o = _pf_only(oracle_mod, shape, phis, [body(fixed=1) for _ in range(3)], kinetics=1, motion=0,
                 mobility=0.02, repulsion=0)
    for _ in range(5):
        o.step(10)
        p = o.phi()
        assert p.min() >= 0.0 and p.max() <= 1.0
        assert p.sum(0).max() <= 1.0 + 1e-15


def test_kinetics_volume_restoring_term_bounds_shrinkage(oracle_mod):
    """A diffuse sphere shrinks under curvature-driven kinetics.  The driving force
    dg = (4 eta / pi^2) dV / |interface| (Sec. 3.3) feeds the volume deficit back, so the deficit
    levels off, while the same run with the term suppressed (emulated by restarting every step,
    so the reference volume always equals the current one) keeps losing volume."""
    shape = (20, 20, 20)
    phi = sphere_phi(shape, (9.5, 10.0, 10.5), 5.0, 5.0)[None]
    o = _pf_only(oracle_mod, shape, phi, [body(fixed=1)], kinetics=1, motion=0, mobility=0.05)
    v0 = phi.sum()
    o.step(100)
    with_term_100 = v0 - o.phi().sum()
    o.step(100)
    with_term_200 = v0 - o.phi().sum()
    cur = phi.copy()
    free = []
    for n in range(200):
        q = _pf_only(oracle_mod, shape, cur, [body(fixed=1)], kinetics=1, motion=0, mobility=0.05)
        q.step(1)
        cur = q.phi()
        if n in (99, 199):
            free.append(v0 - cur.sum())
    growth_free = free[1] - free[0]
    growth_term = with_term_200 - with_term_100
    assert growth_free > 0.0
    assert abs(growth_term) < 0.2 * growth_free
