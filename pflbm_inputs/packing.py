"""Seeded random packings of polydisperse spheres in a periodic cube."""
from __future__ import annotations

import math

import numpy as np


def random_packing(n: int = 1000, r_min: float = 12.0, r_max: float = 18.0, solid_fraction: float = 0.30,
                   min_gap: float = 0.5, seed: int = 0, max_tries: int = 200000):
    """Random sequential addition (PCG64): radii U[r_min, r_max], placed largest first at uniform
    random positions, a position accepted when every surface gap (minimum image) is at least
    min_gap; the cube edge is set by the solid volume fraction.  Returns (centres [n][3],
    radii [n], edge)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    radii = np.sort(rng.uniform(r_min, r_max, n))[::-1].copy()
    L = (float((4.0 / 3.0 * math.pi * radii ** 3).sum()) / solid_fraction) ** (1.0 / 3.0)
    x = np.empty((n, 3))
    tries = 0
    for i in range(n):
        while True:
            tries += 1
            if tries > max_tries:
                raise RuntimeError("random_packing: solid fraction too high for sequential addition")
            c = rng.uniform(0.0, L, 3)
            if i:
                d = x[:i] - c
                d -= L * np.floor(d / L + 0.5)
                if (np.sqrt((d * d).sum(axis=1)) - radii[:i] - radii[i]).min() < min_gap:
                    continue
            x[i] = c
            break
    return x, radii, L
