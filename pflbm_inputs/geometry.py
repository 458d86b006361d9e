"""Rasterisation of diffuse solid bodies and liquid regions on a periodic lattice.

Cell centres sit at integer coordinates; arrays are indexed [z, y, x] (x fastest in memory).
A diffuse indicator is phi = (1 - tanh(2 d / W)) / 2 with d the signed distance to the nominal
surface (positive outside) and W the profile width.  Values within 1e-2 of 0 or 1 are snapped
so that the support of every phase field and its interface set are finite (a 1e-3 snap would
leave the tails of a width-4 plate profile wrapping around a 32-cell periodic box).
"""
from __future__ import annotations

import numpy as np

SNAP = 1e-2


def grid(shape):
    """Cell-centre coordinates x, y, z as read-only full-shape broadcast views."""
    nz, ny, nx = shape
    return (np.broadcast_to(np.arange(nx, dtype=np.float64)[None, None, :], shape),
            np.broadcast_to(np.arange(ny, dtype=np.float64)[None, :, None], shape),
            np.broadcast_to(np.arange(nz, dtype=np.float64)[:, None, None], shape))


def mimg(d, L):
    return d - L * np.floor(d / L + 0.5)


def tanh_profile(d, width: float):
    return 0.5 * (1.0 - np.tanh(2.0 * np.asarray(d, dtype=np.float64) / width))


def snap(phi, eps: float = SNAP):
    p = np.array(phi, dtype=np.float64, copy=True)
    p[p < eps] = 0.0
    p[p > 1.0 - eps] = 1.0
    return p


def box_signed_distance(shape, lo, hi):
    """Signed distance to the axis-aligned box [lo, hi] (continuous coordinates), periodic
    minimum image about the box centre; negative inside."""
    x, y, z = grid(shape)
    nz, ny, nx = shape
    c = [(lo[i] + hi[i]) / 2.0 for i in range(3)]
    h = [(hi[i] - lo[i]) / 2.0 for i in range(3)]
    q = [np.abs(mimg(x - c[0], nx)) - h[0], np.abs(mimg(y - c[1], ny)) - h[1], np.abs(mimg(z - c[2], nz)) - h[2]]
    outside = np.sqrt(sum(np.maximum(qi, 0.0) ** 2 for qi in q))
    inside = np.minimum(np.maximum(np.maximum(q[0], q[1]), q[2]), 0.0)
    return outside + inside


def sphere_signed_distance(shape, centre, radius):
    nz, ny, nx = shape
    # per-axis minimum images, summed x + y + z in that order
    dx = mimg(np.arange(nx, dtype=np.float64) - centre[0], nx) ** 2
    dy = mimg(np.arange(ny, dtype=np.float64) - centre[1], ny) ** 2
    dz = mimg(np.arange(nz, dtype=np.float64) - centre[2], nz) ** 2
    r = np.sqrt((dx[None, None, :] + dy[None, :, None]) + dz[:, None, None])
    return r - radius


def plate_phi(shape, core_lo, core_hi, width: float = 4.0):
    """A plate whose solid-node core is the cells core_lo..core_hi (inclusive integer bounds).
    The nominal surface is offset 3 cells outside the core faces so that, with width 4, core
    cells have phi >= 0.970 and every other cell phi < 0.95: the solid nodes are the core."""
    lo = [core_lo[i] - 0.5 for i in range(3)]
    hi = [core_hi[i] + 0.5 for i in range(3)]
    d = box_signed_distance(shape, lo, hi)
    return snap(tanh_profile(d - 3.0, width))


def _axis_window(n, c, h):
    """Indices of the cells within h of coordinate c on a periodic axis of n cells (all cells when
    the window would wrap onto itself)."""
    lo, hi = int(np.floor(c - h)), int(np.ceil(c + h))
    if hi - lo + 1 >= n:
        return np.arange(n)
    return np.arange(lo, hi + 1) % n


def sphere_phi(shape, centre, radius, width: float = 4.0, out=None):
    """snap(tanh_profile(sphere_signed_distance)), evaluated on the cells within radius + 2 width
    + 1 of the centre per axis: beyond 2 width outside the surface the profile is below 3.4e-4 and
    snaps to exactly 0, so the result is the same array as the whole-grid evaluation.  out: a
    zero-filled array of the grid's shape to write into (returned)."""
    nz, ny, nx = shape
    h = radius + 2.0 * width + 1.0
    ix, iy, iz = (_axis_window(n, c, h) for n, c in ((nx, centre[0]), (ny, centre[1]), (nz, centre[2])))
    dx = mimg(ix.astype(np.float64) - centre[0], nx) ** 2
    dy = mimg(iy.astype(np.float64) - centre[1], ny) ** 2
    dz = mimg(iz.astype(np.float64) - centre[2], nz) ** 2
    d = np.sqrt((dx[None, None, :] + dy[None, :, None]) + dz[:, None, None]) - radius
    if out is None:
        out = np.zeros(shape)
    out[np.ix_(iz, iy, ix)] = snap(tanh_profile(d, width))
    return out


def liquid_density(d_liquid, rho_l: float, rho_v: float, width: float = 4.0):
    """rho = rho_v + (rho_l - rho_v) * (1 - tanh(2 d / W)) / 2, d = signed distance to the
    liquid region (positive in the vapour)."""
    return rho_v + (rho_l - rho_v) * tanh_profile(d_liquid, width)


_M64 = (1 << 64) - 1


def splitmix64_uniform(seed: int, stream: int, n, lo: float, hi: float) -> np.ndarray:
    """Counter-based uniforms in [lo, hi): SplitMix64 (Steele, Lea, Flood 2014) applied to the
    counter seed * 2^40 + stream * 2^32 + k, k = 0..n-1 (or k = the entries of n when n is an
    array of counters); top 53 bits as the mantissa."""
    with np.errstate(over="ignore"):
        k = np.asarray(n, dtype=np.uint64) if np.ndim(n) else np.arange(n, dtype=np.uint64)
        base = np.uint64(((seed << 40) + (stream << 32)) & _M64)
        z = (base + k) * np.uint64(0x9E3779B97F4A7C15) + np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    u = (z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)
    return lo + (hi - lo) * u
