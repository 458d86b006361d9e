"""Liquid/vapour densities used to initialise the two-phase fluid.

For the pseudopotential fluid of Sec. 3.2.3 the bulk equation of state is
p = c_s^2 rho + c_s^2 G psi^2 / 2 with psi = 1 - exp(-rho/rho0).  At G = -5 the paper's parameter
table (Sec. 3.3) gives the liquid density 1.888; the vapour density is the other root of equal
bulk pressure, p(rho_v) = p(1.888).  For other couplings the continuum equal-area rule in the
measure dpsi/psi^2 (Shan & Chen 1993; Shan 2008) is used.  These are initial values only.
"""
from __future__ import annotations

import math
from functools import lru_cache

from scipy import integrate, optimize

CS2 = 1.0 / 3.0
PAPER_RHO_L = 1.888  # liquid density at G = -5, rho0 = 1 (parameter table, Sec. 3.3)


def _eos(G, rho0):
    def psi(r):
        return 1.0 - math.exp(-r / rho0)

    def p(r):
        return CS2 * r + 0.5 * CS2 * G * psi(r) ** 2

    return psi, p


def vapour_for_liquid(rho_l: float, G: float = -5.0, rho0: float = 1.0) -> float:
    """Vapour-branch density with the same bulk pressure as rho_l."""
    _, p = _eos(G, rho0)
    target = p(rho_l)
    # the vapour branch rises from 0 to the first pressure maximum
    rmax = optimize.minimize_scalar(lambda r: -p(r), bounds=(1e-6, rho_l), method="bounded").x
    return float(optimize.brentq(lambda r: p(r) - target, 1e-9, rmax, xtol=1e-15))


@lru_cache(maxsize=32)
def equal_area_densities(G: float = -5.0, rho0: float = 1.0) -> tuple:
    """(rho_v, rho_l) from the continuum pseudopotential equal-area rule."""
    if G >= -4.0:  # critical coupling of psi = 1 - exp(-rho/rho0) is G_c = -4
        raise ValueError("no phase separation for G >= -4")
    psi, p = _eos(G, rho0)

    def dpsi(r):
        return math.exp(-r / rho0) / rho0

    def eqs(v):
        rv, rl = v
        p0 = p(rv)
        area, _ = integrate.quad(lambda r: (p0 - p(r)) * dpsi(r) / psi(r) ** 2, rv, rl, epsabs=1e-14, epsrel=1e-13)
        return [p(rl) - p0, area]

    rv, rl = optimize.fsolve(eqs, [0.15, 1.9], xtol=1e-14)
    return float(rv), float(rl)


@lru_cache(maxsize=32)
def coexistence_densities(G: float = -5.0, rho0: float = 1.0) -> tuple:
    """(rho_vapour, rho_liquid) for initial fields."""
    if G == -5.0 and rho0 == 1.0:
        return vapour_for_liquid(PAPER_RHO_L, G, rho0), PAPER_RHO_L
    return equal_area_densities(G, rho0)
