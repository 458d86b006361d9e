"""Parameter sets.

The defaults follow the parameter table of Sec. 3.3 of the paper (rho0 = 1, tau = 1.1,
G = -5, wetting parameter 2.0, phase-field mobility 1e-5, interface width 5), the solid
threshold of Sec. 3.2.2 (0.05 on the fluid fraction), the repulsion range and exponent of
Sec. 3.1.2 (r_c = 3 dx, n = 4) and the redistribution radius R_A = dx of Sec. 3.2.2.

Values the paper does not give are readings:
  * sigma_ab: solid/fluid 1.0, solid/solid 0.5 (grain-boundary energy below the surface
    energy, Sec. 4.3.1); units folded into the mobility.
  * e0 (repulsion strength): 0.05.
  * the named workloads run tau = 1.0 on a D3Q19 lattice (Sec. 3.2.1 prints D3Q27, which is
    available as lattice = 27).
"""
from __future__ import annotations

import numpy as np

# Resolution of "phi > 0" in the present-phase and interface sets of Sec. 3.3 (a reading): phase
# values at or below the unit round-off of FP64, 2^-53, cannot change the fluid fraction
# 1 - sum phi and count as absent.
PHI_FLOOR = 2.0 ** -53


def sigma_matrix(nb: int, sigma_sf: float = 1.0, sigma_ss: float = 0.5) -> np.ndarray:
    """(nb+1) x (nb+1) interface energies, phase 0 = fluid, zero diagonal."""
    s = np.full((nb + 1, nb + 1), sigma_ss, dtype=np.float64)
    s[0, :] = sigma_sf
    s[:, 0] = sigma_sf
    np.fill_diagonal(s, 0.0)
    return s


def paper_params(nx: int, ny: int, nz: int, nb: int) -> dict:
    return {
        "nx": nx, "ny": ny, "nz": nz,
        "tau": 1.1, "G": -5.0, "rho0": 1.0,
        "solid_threshold": 0.05,
        "mobility": 1e-5, "eta": 5.0,
        "sigma": sigma_matrix(nb),
        "rc": 3.0, "nexp": 4.0, "e0": 0.05,
        "RA": 1.0,
        "fext": (0.0, 0.0, 0.0),
        "kinetics": 1, "motion": 1, "repulsion": 1,
        "lattice": 19,
        "phi_floor": PHI_FLOOR,
    }


def default_params(nx: int, ny: int, nz: int, nb: int, **over) -> dict:
    """Paper parameters with tau = 1.0 (the value the named workloads run)."""
    p = paper_params(nx, ny, nz, nb)
    p["tau"] = 1.0
    for k, v in over.items():
        if k not in p:
            raise KeyError(k)
        p[k] = v
    return p
