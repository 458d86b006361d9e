"""Helpers for the oracle pin tests: builds small inputs and reads totals.  No arithmetic of
the method lives here; closed forms used as expectations are derived in each test."""
import numpy as np

from pflbm_inputs import default_params


def empty_fluid(shape):
    return np.zeros(shape)


def slab_phi(shape, z_layers):
    """One sharp solid layer set (phi = 1 on the given z planes, 0 elsewhere)."""
    p = np.zeros(shape)
    for z in z_layers:
        p[z] = 1.0
    return p


def params(shape, nb, **over):
    nz, ny, nx = shape
    return default_params(nx, ny, nz, nb, **over)


def body(v=(0, 0, 0), w=(0, 0, 0), fixed=1, mass_density=1.0, wet=1.0):
    return {"mass_density": mass_density, "wetting_rho": wet, "v": v, "w": w, "fixed": fixed}


def total_momentum(o):
    j = o.mom().reshape(3, -1).sum(axis=1)
    b = o.bodies()
    c = o.body_consts()
    pb = (c["M"][:, None] * b["V"]).sum(axis=0) if o.nb else np.zeros(3)
    return j + pb
