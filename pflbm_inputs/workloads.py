"""Named synthetic workloads (initial fields + parameters) for the coupled step.

  plates_bridge       two finite plates (solid cores 16x16x2, faces 8 cells apart) joined by a
                      liquid cylinder of radius 6, 32^3, 90 degree wetting; the paper's plate
                      benchmark of Sec. 4.2 at dx/R = 1/6.
  two_spheres_bridge  two spheres R = 20 (nominal surface gap 4) in 128^3 with a liquid bridge of
                      2 % of one sphere's volume, 30 degree wetting; Sec. 4.3.1 scaled to R = 20.
  tetrahedron_drop    four spheres R = 24 at the vertices of a regular tetrahedron (edge 2R + 4) in
                      256^3 with a central drop of 5 % liquid fraction and seeded 1e-3 perturbations
                      of the phase fields; Sec. 4.3.2 scaled to R = 24.
  tiny_moving_body    small ragged grids with a moving, rotating sphere and a drop, for parity and
                      invariant tests (node conversion, moving-wall bounce-back).

The paper's figures hold no data in the available text, so these inputs stand in for its
experiments; none reproduces a published curve.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from .coexistence import coexistence_densities
from .geometry import grid, liquid_density, mimg, plate_phi, snap, sphere_phi, splitmix64_uniform
from .params import default_params

PLATE_DENSITY_RATIO = 1.72e4   # rho_S / rho_L for the plate tests (Sec. 4.2)
SPHERE_DENSITY = 4.0           # sphere mass density (Sec. 4.3)


# Wetting parameter varrho_B against contact angle (degrees) at G = -5, rho0 = 1, tau = 1,
# measured with the oracle on the planar capillary bridge through the Young-Laplace law
# (tests/golden/calibrate_wetting.py writes tests/golden/wetting_calibration.json).
WETTING_TABLE = ((0.0, 1.3542), (30.0, 1.2280), (60.0, 0.9690), (90.0, 0.7067))


def wetting_rho_for_angle(theta_deg: float, G: float = -5.0, rho0: float = 1.0) -> float:
    """Wetting parameter varrho_B for a contact angle in [0, 90] degrees: the calibrated table,
    linear in cos(theta) between its points (the paper defers this map to Benzi et al. 2006).
    The table holds for G = -5, rho0 = 1 only."""
    if G != -5.0 or rho0 != 1.0:
        raise ValueError("the wetting table is calibrated for G = -5, rho0 = 1")
    if not 0.0 <= theta_deg <= 90.0:
        raise ValueError("contact angles in [0, 90] degrees only")
    c = math.cos(math.radians(theta_deg))
    pts = [(math.cos(math.radians(t)), w) for t, w in WETTING_TABLE]
    for (c0, w0), (c1, w1) in zip(pts, pts[1:]):
        if c1 <= c <= c0:
            return w0 + (w1 - w0) * (c - c0) / (c1 - c0)
    return pts[-1][1]


@dataclass
class Workload:
    name: str
    params: dict
    bodies: list
    rho0: np.ndarray            # [nz, ny, nx] float64
    phi0: np.ndarray            # [nb, nz, ny, nx] float64
    meta: dict = field(default_factory=dict)

    @property
    def shape(self):
        return self.rho0.shape

    @property
    def cells(self) -> int:
        return int(self.rho0.size)


def _body(mass_density, wetting_rho, v=(0, 0, 0), w=(0, 0, 0), fixed=0):
    return {"mass_density": float(mass_density), "wetting_rho": float(wetting_rho),
            "v": tuple(float(a) for a in v), "w": tuple(float(a) for a in w), "fixed": int(fixed)}


def _solid_mask(phi0, threshold=0.05):
    return (1.0 - phi0.sum(axis=0)) < threshold if phi0.shape[0] else np.zeros(phi0.shape[1:], bool)


def _liquid_volume(rho, solid, rv, rl):
    """Liquid volume counted on fluid nodes as clamp((rho - rho_v)/(rho_l - rho_v), 0, 1)."""
    frac = np.clip((rho - rv) / (rl - rv), 0.0, 1.0)
    return float(frac[~solid].sum())


def _bisect(fn, lo, hi, target, iters=50):
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        if fn(mid) < target:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def uniform_fluid(shape=(8, 8, 8), rho=1.0, **over):
    nz, ny, nx = shape
    p = default_params(nx, ny, nz, 0, **over)
    return Workload("uniform_fluid", p, [], np.full(shape, float(rho)), np.zeros((0,) + tuple(shape)))


def plates_bridge(n: int = 32, radius: float = 6.0, gap: int = 8, plate: int = 16, thickness: int = 2,
                  width: float = 4.0, theta_deg: float = 90.0, fixed: bool = False, **over) -> Workload:
    """Two finite parallel plates joined by a cylindrical liquid bridge (Sec. 4.2)."""
    shape = (n, n, n)
    rv, rl = coexistence_densities()
    lo = (n - plate) // 2
    hi = lo + plate - 1
    zc = n / 2.0 - 0.5                            # mirror plane between the plates
    z_top_lo = int(round(zc + gap / 2.0 + 0.5))   # first solid layer of the upper plate
    z_bot_hi = int(round(zc - gap / 2.0 - 0.5))   # last solid layer of the lower plate
    phis = np.stack([
        plate_phi(shape, (lo, lo, z_bot_hi - thickness + 1), (hi, hi, z_bot_hi), width),
        plate_phi(shape, (lo, lo, z_top_lo), (hi, hi, z_top_lo + thickness - 1), width),
    ])
    x, y, z = grid(shape)
    cx = cy = (lo + hi) / 2.0
    r = np.sqrt(mimg(x - cx, n) ** 2 + mimg(y - cy, n) ** 2)
    # liquid cylinder bounded by the plates' solid faces
    dz = np.abs(z - zc) - gap / 2.0
    d = np.maximum(r - radius, dz)
    rho = liquid_density(d, rl, rv, width)
    wet = wetting_rho_for_angle(theta_deg)
    ms = PLATE_DENSITY_RATIO * rl
    bodies = [_body(ms, wet, fixed=int(fixed)), _body(ms, wet, fixed=int(fixed))]
    p = default_params(n, n, n, 2, **over)
    meta = {"radius": radius, "gap": gap, "rho_l": rl, "rho_v": rv, "theta_deg": theta_deg,
            "plate_cells": plate * plate * thickness, "z_faces": (z_bot_hi + 0.5, z_top_lo - 0.5)}
    return Workload("plates_bridge", p, bodies, rho, phis, meta)


def planar_bridge(nx: int = 80, nz: int = 50, gap: int = 20, plate: int = 48, thickness: int = 2,
                  liquid_width: float = 28.0, width: float = 4.0, wetting_rho: float | None = None,
                  theta_deg: float = 90.0, **over) -> Workload:
    """Planar capillary bridge (Sec. 2.1.1, planar case): two finite plates, ``plate`` cells long
    in x and infinite in y (ny = 1), solid faces ``gap`` cells apart, joined by a liquid slab
    ``liquid_width`` cells wide; vapour all around.  The plates are held fixed."""
    shape = (nz, 1, nx)
    rv, rl = coexistence_densities()
    x, y, z = grid(shape)
    zc, xc = nz / 2.0 - 0.5, nx / 2.0 - 0.5
    z_bot_hi = int(round(zc - gap / 2.0 - 0.5))
    z_top_lo = int(round(zc + gap / 2.0 + 0.5))
    x0 = int(round(xc - plate / 2.0 + 0.5))
    x1 = x0 + plate - 1
    phis = np.stack([
        plate_phi(shape, (x0, 0, z_bot_hi - thickness + 1), (x1, 0, z_bot_hi), width),
        plate_phi(shape, (x0, 0, z_top_lo), (x1, 0, z_top_lo + thickness - 1), width),
    ])
    d = np.maximum(np.abs(x - xc) - liquid_width / 2.0, np.abs(z - zc) - gap / 2.0)
    rho = liquid_density(d, rl, rv, width)
    wet = wetting_rho_for_angle(theta_deg) if wetting_rho is None else float(wetting_rho)
    ms = PLATE_DENSITY_RATIO * rl
    bodies = [_body(ms, wet, fixed=1), _body(ms, wet, fixed=1)]
    over.setdefault("motion", 0)
    p = default_params(nx, 1, nz, 2, **over)
    meta = {"gap": gap, "rho_l": rl, "rho_v": rv, "wetting_rho": wet, "z_mid": int(round(zc)),
            "x_centre": int(round(xc)), "z_faces": (z_bot_hi + 0.5, z_top_lo - 0.5)}
    return Workload("planar_bridge", p, bodies, rho, phis, meta)


def two_spheres_bridge(n: int = 128, radius: float = 20.0, gap: float = 4.0, liquid_fraction: float = 0.02,
                       theta_deg: float = 30.0, width: float = 4.0, **over) -> Workload:
    """Two equal spheres joined by a liquid bridge whose volume is a fraction of one sphere's
    volume, placed as a tanh-smoothed cylinder along the line of centres (Sec. 4.3.1)."""
    shape = (n, n, n)
    rv, rl = coexistence_densities()
    c = n / 2.0
    half = radius + gap / 2.0
    centres = [(c - half, c, c), (c + half, c, c)]
    phis = np.stack([sphere_phi(shape, ctr, radius, width) for ctr in centres])
    solid = _solid_mask(phis)
    x, y, z = grid(shape)
    rperp = np.sqrt(mimg(y - c, n) ** 2 + mimg(z - c, n) ** 2)
    dx = np.abs(mimg(x - c, n)) - half
    target = liquid_fraction * 4.0 / 3.0 * math.pi * radius ** 3

    def vol(rb):
        return _liquid_volume(liquid_density(np.maximum(rperp - rb, dx), rl, rv, width), solid, rv, rl)

    rb = _bisect(vol, 0.5, radius, target)
    rho = liquid_density(np.maximum(rperp - rb, dx), rl, rv, width)
    wet = wetting_rho_for_angle(theta_deg)
    bodies = [_body(SPHERE_DENSITY, wet), _body(SPHERE_DENSITY, wet)]
    p = default_params(n, n, n, 2, **over)
    meta = {"radius": radius, "gap": gap, "bridge_radius": rb, "liquid_volume": vol(rb), "target_volume": target,
            "rho_l": rl, "rho_v": rv, "theta_deg": theta_deg, "centres": centres}
    return Workload("two_spheres_bridge", p, bodies, rho, phis, meta)


def bridge_pair(shape, r1: float, r2: float, gap: float, liquid_fraction: float, theta_deg: float,
                width: float = 4.0, rho_v_init: float | None = None, fixed: bool = False, **over) -> Workload:
    """Two spheres of radii r1, r2 on the x axis with a surface gap, joined by a tanh-smoothed
    cylindrical bridge of liquid volume V_L = c V_S / (1 - c), c the liquid fraction
    V_L / (V_L + V_S) of Sec. 2.2 and V_S the two spheres' volume; the bridge radius is found by
    bisection (capped at the smaller radius).  rho_v_init, when given, replaces the flat-interface
    vapour density as the initial vapour (BRIDGE_VAPOUR gives the reason).  fixed holds both
    spheres in place (the rigid-body update leaves them at rest)."""
    nz, ny, nx = shape
    rv, rl = coexistence_densities()
    if rho_v_init is not None:
        rv = float(rho_v_init)
    cy, cz = ny / 2.0, nz / 2.0
    c1 = (nx / 2.0 - gap / 2.0 - r1, cy, cz)
    c2 = (nx / 2.0 + gap / 2.0 + r2, cy, cz)
    phis = np.stack([sphere_phi(shape, c1, r1, width), sphere_phi(shape, c2, r2, width)])
    tot = phis.sum(0)
    phis = np.where(tot > 1.0, phis / np.where(tot > 1.0, tot, 1.0), phis)
    solid = _solid_mask(phis)
    # the bridge lives in a window around the segment between the centres
    m = int(math.ceil(2 * width)) + 1
    x0, x1 = max(int(c1[0]) - m, 0), min(int(math.ceil(c2[0])) + m + 1, nx)
    rr = int(math.ceil(min(r1, r2))) + m
    y0, y1 = max(int(cy) - rr, 0), min(int(cy) + rr + 1, ny)
    z0, z1 = max(int(cz) - rr, 0), min(int(cz) + rr + 1, nz)
    x, y, z = grid(shape)
    win = (slice(z0, z1), slice(y0, y1), slice(x0, x1))
    xm = 0.5 * (c1[0] + c2[0])
    half = 0.5 * (c2[0] - c1[0])
    rperp_w = np.sqrt((y[win] - cy) ** 2 + (z[win] - cz) ** 2)
    dx_w = np.abs(x[win] - xm) - half
    solid_w = solid[win]
    target = liquid_fraction / (1.0 - liquid_fraction) * 4.0 / 3.0 * math.pi * (r1 ** 3 + r2 ** 3)

    def vol(rb):
        return _liquid_volume(liquid_density(np.maximum(rperp_w - rb, dx_w), rl, rv, width), solid_w, rv, rl)

    rmax = min(r1, r2)
    rb = rmax if vol(rmax) < target else _bisect(vol, 0.5, rmax, target, iters=30)
    rperp = np.sqrt((y - cy) ** 2 + (z - cz) ** 2)
    rho = liquid_density(np.maximum(rperp - rb, np.abs(x - xm) - half), rl, rv, width)
    wet = wetting_rho_for_angle(theta_deg)
    bodies = [_body(SPHERE_DENSITY, wet, fixed=int(fixed)), _body(SPHERE_DENSITY, wet, fixed=int(fixed))]
    p = default_params(nx, ny, nz, 2, **over)
    meta = {"radii": (r1, r2), "gap": gap, "liquid_fraction": liquid_fraction, "theta_deg": theta_deg,
            "bridge_radius": rb, "liquid_volume": vol(rb), "target_volume": target, "centres": (c1, c2),
            "rho_l": rl, "rho_v": rv}
    return Workload("bridge_pair", p, bodies, rho, phis, meta)


def bridge_sweep_params(n: int = 64, seed: int = 0, min_len: int = 48, max_len: int = 128):
    """Seeded parameters of a sweep of uneven two-sphere bridges (PCG64): radii U[8, 30], surface gap
    U[2, 8], liquid fraction U[0.01, 0.20], contact angle U[0, 60] degrees; box length per axis
    U[min_len, max_len] rounded up to a multiple of 8, redrawn until the pair fits with 8 cells
    to spare on every side (x: 2 r1 + 2 r2 + gap + 16; y, z: 2 max(r) + 16)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    while len(out) < n:
        r1, r2 = rng.uniform(8.0, 30.0, 2)
        gap = rng.uniform(2.0, 8.0)
        c = rng.uniform(0.01, 0.20)
        theta = rng.uniform(0.0, 60.0)
        L = [int(math.ceil(v / 8.0) * 8) for v in rng.uniform(min_len, max_len, 3)]
        if L[0] < 2 * (r1 + r2) + gap + 16 or min(L[1], L[2]) < 2 * max(r1, r2) + 16 or max(L) > max_len:
            continue
        out.append({"shape": (L[2], L[1], L[0]), "r1": float(r1), "r2": float(r2), "gap": float(gap),
                    "liquid_fraction": float(c), "theta_deg": float(theta)})
    return out


def bridge_sweep(n: int = 64, seed: int = 0, **over) -> list:
    """The sweep of bridge_sweep_params as workloads."""
    return [bridge_pair(q["shape"], q["r1"], q["r2"], q["gap"], q["liquid_fraction"], q["theta_deg"], **over)
            for q in bridge_sweep_params(n, seed)]


# Initial vapour density of isolated two-sphere bridges in large vapour boxes.  Sec. 2 neglects
# evaporation and takes the liquid volume as constant.  In the pseudopotential fluid, wetting
# spheres started in vapour at the flat-interface density (0.119) draw the liquid of small bridges
# into adsorbed layers on their surfaces: bridges below about 8000 liquid cells drain to zero
# force within about 1000 steps in boxes of 48^3..128^3.  Started at 0.136 (measured, two-sphere
# sweep and 96^3 pairs, theta 0..60 degrees), bridges down to about 800 cells at gaps up to about
# 4 cells keep their force over 2000 steps, the force of large bridges moves by under 10 %, and
# no bridge condenses between spheres without liquid; thin bridges across wider gaps still break.
BRIDGE_VAPOUR = 0.136


def tetrahedron_drop(n: int = 256, radius: float = 24.0, gap: float = 4.0, liquid_fraction: float = 0.05,
                     theta_deg: float = 30.0, width: float = 4.0, seed: int = 0, amplitude: float = 1e-3,
                     **over) -> Workload:
    """Four spheres at the vertices of a regular tetrahedron with a central liquid drop; liquid
    fraction c = V_L / (V_L + V_S); seeded uniform perturbations on the interface cells of every
    phase field, then clip and renormalise (Sec. 4.3.2).  Runs at the paper's tau = 1.1 (the
    parameter table of Sec. 3.3) unless tau is given."""
    over.setdefault("tau", 1.1)
    shape = (n, n, n)
    rv, rl = coexistence_densities()
    c = n / 2.0
    edge = 2.0 * radius + gap
    circ = edge * math.sqrt(6.0) / 4.0
    verts = np.array([(1, 1, 1), (1, -1, -1), (-1, 1, -1), (-1, -1, 1)], dtype=np.float64) / math.sqrt(3.0) * circ
    centres = [tuple(c + v) for v in verts]
    phis = np.zeros((len(centres),) + shape)
    for a, ctr in enumerate(centres):
        sphere_phi(shape, ctr, radius, width, out=phis[a])
    for a in range(phis.shape[0]):
        band = (phis[a] > 0.0) & (phis[a] < 1.0)
        idx = np.flatnonzero(band.reshape(-1))
        # the uniform of counter k (the cell's flat index) for the band cells only
        flat = phis[a].reshape(-1)
        flat[idx] += splitmix64_uniform(seed, a, idx, -amplitude, amplitude)
    phis = np.clip(phis, 0.0, 1.0)
    tot = phis.sum(axis=0)
    over1 = tot > 1.0
    phis[:, over1] /= tot[over1]
    solid = _solid_mask(phis)
    x, y, z = grid(shape)
    rr = np.sqrt(mimg(x - c, n) ** 2 + mimg(y - c, n) ** 2 + mimg(z - c, n) ** 2)
    vs = 4 * 4.0 / 3.0 * math.pi * radius ** 3
    target = liquid_fraction / (1.0 - liquid_fraction) * vs
    # the drop's profile reaches the vapour density exactly (tanh rounds to 1 in FP64) 9.5 widths
    # outside its surface, so the bisection sums the liquid volume over the cube around the
    # centre that holds every drop radius it tries
    win = np.arange(n) if circ + 10.0 * width + 1.0 >= n / 2.0 else \
        np.arange(int(np.floor(c - circ - 10.0 * width - 1.0)), int(np.ceil(c + circ + 10.0 * width + 1.0)) + 1) % n
    sub = np.ix_(win, win, win)
    rr_w, solid_w = rr[sub], solid[sub]

    def vol(rd):
        return _liquid_volume(liquid_density(rr_w - rd, rl, rv, width), solid_w, rv, rl)

    rd = _bisect(vol, 1.0, circ, target)
    rho = liquid_density(rr - rd, rl, rv, width)
    wet = wetting_rho_for_angle(theta_deg)
    bodies = [_body(SPHERE_DENSITY, wet) for _ in centres]
    p = default_params(n, n, n, 4, **over)
    meta = {"radius": radius, "edge": edge, "drop_radius": rd, "liquid_volume": vol(rd), "target_volume": target,
            "rho_l": rl, "rho_v": rv, "seed": seed, "amplitude": amplitude, "centres": centres}
    return Workload("tetrahedron_drop", p, bodies, rho, phis, meta)


def tiny_moving_body(shape=(10, 12, 14), radius: float = 3.2, v=(0.05, -0.03, 0.02), w=(0.0, 0.0, 0.01),
                     second_body: bool = False, drop: bool = True, width: float = 2.0, **over) -> Workload:
    """A small ragged grid with a moving, rotating sphere (and optionally a second, resting one
    close to it) next to a liquid drop; exercises moving-wall bounce-back, node conversion,
    repulsion and the phase-field update on a grid small enough for exhaustive comparison."""
    nz, ny, nx = shape
    rv, rl = coexistence_densities()
    centres = [(nx * 0.35, ny * 0.5, nz * 0.5)]
    if second_body:
        centres.append((centres[0][0] + 2 * radius + 0.7, ny * 0.5 + 0.4, nz * 0.5 - 0.3))
    phis = np.stack([sphere_phi(shape, ctr, radius, width) for ctr in centres])
    x, y, z = grid(shape)
    if drop:
        dc = (nx * 0.8, ny * 0.45, nz * 0.55)
        d = np.sqrt(mimg(x - dc[0], nx) ** 2 + mimg(y - dc[1], ny) ** 2 + mimg(z - dc[2], nz) ** 2) - 2.5
        rho = liquid_density(d, rl, rv, width)
    else:
        rho = np.full(shape, rv)
    bodies = [_body(SPHERE_DENSITY, 1.4, v=v, w=w)]
    if second_body:
        bodies.append(_body(SPHERE_DENSITY, 1.1))
    p = default_params(nx, ny, nz, len(bodies), **over)
    return Workload("tiny_moving_body", p, bodies, rho, phis, {"centres": centres})


WORKLOADS = {
    "planar_bridge": planar_bridge,
    "plates_bridge": plates_bridge,
    "two_spheres_bridge": two_spheres_bridge,
    "tetrahedron_drop": tetrahedron_drop,
    "tiny_moving_body": tiny_moving_body,
    "uniform_fluid": uniform_fluid,
}


def make_workload(name: str, **kw) -> Workload:
    return WORKLOADS[name](**kw)
