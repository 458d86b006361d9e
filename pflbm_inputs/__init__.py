"""Seeded, synthetic inputs for the coupled phase-field / lattice-Boltzmann step.

This module generates initial conditions only: phase-field rasterisations of plates and spheres
with diffuse (tanh) profiles, liquid/vapour density fields, parameter sets and the named
workloads, and random sphere packings.  It holds none of the time step's arithmetic, and it is the
only code shared by the CPU oracle's tests and the GPU library's tests, benchmark, smoke check and
the surrogate pipeline (which builds the initial conditions of its field re-solves here).
"""
from .params import default_params, paper_params, sigma_matrix  # noqa: F401
from .geometry import (  # noqa: F401
    tanh_profile, snap, box_signed_distance, sphere_signed_distance, plate_phi, sphere_phi,
    liquid_density, splitmix64_uniform,
)
from .coexistence import coexistence_densities  # noqa: F401
from .packing import random_packing  # noqa: F401
from .workloads import (  # noqa: F401
    Workload, planar_bridge, plates_bridge, two_spheres_bridge, bridge_pair, bridge_sweep, bridge_sweep_params, tetrahedron_drop, tiny_moving_body, uniform_fluid,
    BRIDGE_VAPOUR, SPHERE_DENSITY,
    WORKLOADS, make_workload,
)
