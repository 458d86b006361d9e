"""Pins of the oracle's pseudopotential fluid (Sec. 3.2.3) against its own continuum theory:
flat-interface coexistence near the equal-area rule of the pseudopotential equation of state,
equal bulk pressures across a flat interface, the Young-Laplace law (Sec. 2.1.1) for
cylindrical drops, and agreement of the Laplace surface tension with the profile integral of
Sec. 3.2.3 to the ~10 % the paper itself reports between the two (Sec. 4.1)."""
import math

import numpy as np
import pytest

from pflbm_inputs import coexistence_densities, liquid_density, uniform_fluid
from pflbm_inputs.coexistence import equal_area_densities

CS2 = 1.0 / 3.0
G = -5.0


def _pressure(rho):
    psi = 1.0 - np.exp(-rho)
    return CS2 * rho + 0.5 * CS2 * G * psi ** 2


def _slab(oracle_mod, L=64, steps=8000, **over):
    rv, rl = coexistence_densities(G)
    x = np.arange(L)
    d = np.abs(x - (L - 1) / 2.0) - L / 4.0
    rho = liquid_density(d, rl, rv, 4.0).reshape(1, 1, L)
    w = uniform_fluid((1, 1, L), G=G, **over)
    o = oracle_mod.Oracle(w.params, [], rho, w.phi0)
    o.step(steps)
    return o.rho()[0, 0], o


@pytest.mark.parametrize("lattice,tau", [(19, 1.0), (27, 1.1)])
def test_flat_interface_coexistence(oracle_mod, lattice, tau):
    """A flat liquid slab relaxes to the liquid density the paper's parameter table prints for
    G = -5 (1.888, Sec. 3.3), and its two bulks have equal equation-of-state pressure (mechanical
    equilibrium).  The continuum equal-area rule (about 1.93 / 0.156) is only approximate on
    the lattice."""
    r, _ = _slab(oracle_mod, lattice=lattice, tau=tau)
    L = r.size
    rho_l, rho_v = r[L // 2], r[0]
    assert abs(rho_l - 1.888) < 1e-3
    assert abs(_pressure(rho_l) - _pressure(rho_v)) < 1e-6 * _pressure(rho_l)
    rv_ea, rl_ea = equal_area_densities(G)
    assert abs(rho_l / rl_ea - 1) < 0.03


def _drop_dp(oracle_mod, R, n=48, steps=4000, **over):
    rv, rl = coexistence_densities(G)
    y, x = np.meshgrid(np.arange(n, dtype=float), np.arange(n, dtype=float), indexing="ij")
    c = (n - 1) / 2.0
    d = np.sqrt((x - c) ** 2 + (y - c) ** 2) - R
    rho = liquid_density(d, rl, rv, 4.0).reshape(1, n, n)
    w = uniform_fluid((1, n, n), G=G, **over)
    o = oracle_mod.Oracle(w.params, [], rho, w.phi0)
    o.step(steps)
    r = o.rho()[0]
    k = int(round(c))
    return _pressure(r[k, k]) - _pressure(r[0, 0])


@pytest.mark.slow
def test_laplace_law_and_surface_tension(oracle_mod):
    """Pressure jump across cylindrical drops is linear in 1/R (Young-Laplace, Sec. 2.1.1) and its
    slope sigma agrees with the profile integral sigma = -(1/2) c_s^4 G int |d psi/dn|^2 dn of a flat
    interface (Sec. 3.2.3; c_s^4 read for the printed c_x^4) within 15 %; the paper's own two
    estimates differ by about 8 % (Sec. 4.1)."""
    radii = [8.0, 10.0, 12.0, 15.0]
    dps = np.array([_drop_dp(oracle_mod, R) for R in radii])
    inv = 1.0 / np.array(radii)
    A = np.vstack([inv, np.ones_like(inv)]).T
    (slope, icpt), res, *_ = np.linalg.lstsq(A, dps, rcond=None)
    pred = A @ np.array([slope, icpt])
    r2 = 1 - ((dps - pred) ** 2).sum() / ((dps - dps.mean()) ** 2).sum()
    assert r2 > 0.99
    assert abs(icpt) < 0.1 * dps.min()
    sigma_laplace = slope
    r, _ = _slab(oracle_mod)
    psi = 1.0 - np.exp(-r)
    dpsi = 0.5 * (np.roll(psi, -1) - np.roll(psi, 1))
    sigma_profile = -0.5 * CS2 * CS2 * G * (dpsi ** 2).sum() / 2.0  # two interfaces in the slab
    assert 0.02 < sigma_laplace < 0.06
    assert abs(sigma_profile / sigma_laplace - 1) < 0.15
    # the paper's profile-integral value for G = -5 is 3.297e-2 (Sec. 4.1); the flat profile
    # depends on the lattice only through its (shared) second and fourth moments
    assert abs(sigma_profile / 3.297e-2 - 1) < 0.01


@pytest.mark.slow
def test_d3q27_surface_tension_against_the_paper(oracle_mod):
    """On the paper's own lattice and relaxation time (D3Q27, tau = 1.1, G = -5, Sec. 4.1): the
    profile integral of a flat interface gives the paper's 3.297e-2 within 1 %, and the Laplace fit
    of cylindrical drops the paper's 3.583e-2 within 10 % (the paper's two estimates themselves
    differ by 8 %); the two estimates here agree within 3 %."""
    radii = [8.0, 10.0, 12.0, 15.0]
    dps = np.array([_drop_dp(oracle_mod, R, lattice=27, tau=1.1) for R in radii])
    inv = 1.0 / np.array(radii)
    A = np.vstack([inv, np.ones_like(inv)]).T
    (slope, icpt), *_ = np.linalg.lstsq(A, dps, rcond=None)
    r, _ = _slab(oracle_mod, lattice=27, tau=1.1)
    psi = 1.0 - np.exp(-r)
    dpsi = 0.5 * (np.roll(psi, -1) - np.roll(psi, 1))
    sigma_profile = -0.5 * CS2 * CS2 * G * (dpsi ** 2).sum() / 2.0
    assert abs(sigma_profile / 3.297e-2 - 1) < 0.01
    assert abs(slope / 3.583e-2 - 1) < 0.10
    assert abs(sigma_profile / slope - 1) < 0.03
