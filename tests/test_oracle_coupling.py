"""Pins of the oracle's solid-fluid coupling (Sec. 3.2.2, 3.2.3) and rigid-body motion (Sec. 3.1):
exact conservation of fluid mass and of total momentum with moving bodies and node conversions,
mirror symmetry, lattice-translation invariance, repulsion against a brute-force pair sum and
force-free kinematics."""
import math

import numpy as np
import pytest

from oracle_helpers import body, params, total_momentum
from pflbm_inputs import plates_bridge, sphere_phi, tiny_moving_body


def _run(oracle_mod, w, steps):
    o = oracle_mod.Oracle(w.params, w.bodies, w.rho0, w.phi0)
    o.step(steps)
    return o


def test_fluid_mass_exact_with_moving_body_and_conversions(oracle_mod):
    """The moving-wall terms are compensated on the rest population and converted nodes hand
    their content to fluid neighbours, so the fluid mass is constant to round-off."""
    w = tiny_moving_body(v=(0.12, -0.07, 0.05), w=(0.0, 0.0, 0.02))
    o = oracle_mod.Oracle(w.params, w.bodies, w.rho0, w.phi0)
    m0 = o.rho().sum()
    o.step(120)
    d = o.diag()
    assert d["n_f2s"] > 5 and d["n_s2f"] > 5, d
    assert d["lost_mass"] == 0.0
    assert abs(o.rho().sum() - m0) < 1e-13 * m0


def test_total_momentum_conserved_free_bodies(oracle_mod):
    """Fluid momentum plus body momentum is invariant: every force on a body (momentum exchange,
    pseudopotential reaction, repulsion) is the opposite of what the fluid or the other body
    receives.  Two free bodies near contact, a drop, node conversions."""
    w = tiny_moving_body(v=(0.1, 0.03, -0.04), second_body=True)
    w.params["e0"] = 0.5
    o = oracle_mod.Oracle(w.params, w.bodies, w.rho0, w.phi0)
    p0 = total_momentum(o)
    rep = 0.0
    for _ in range(30):
        o.step(3)
        assert np.max(np.abs(total_momentum(o) - p0)) < 1e-12
        rep = max(rep, np.abs(o.force_parts()["rep"]).max())
    assert o.diag()["n_f2s"] > 0
    assert rep > 0.0


def test_plates_mirror_symmetry(oracle_mod):
    """The plate-bridge input is mirror symmetric about the mid-plane and the x, y centre lines:
    forces on the plates are equal and opposite along z, zero along x and y."""
    w = plates_bridge(fixed=True)
    o = _run(oracle_mod, w, 40)
    F = o.bodies()["F"]
    assert abs(F[0, 2] + F[1, 2]) < 1e-12 * abs(F[0, 2])
    assert np.max(np.abs(F[:, :2])) < 1e-12 * abs(F[0, 2])
    r = o.rho()
    assert np.max(np.abs(r - r[::-1, :, :])) < 1e-12
    assert np.max(np.abs(r - r[:, ::-1, :])) < 1e-12
    assert np.max(np.abs(r - np.transpose(r, (0, 2, 1)))) < 1e-12


def test_lattice_translation_invariance(oracle_mod):
    """Rolling the whole input by integer offsets rolls every output and shifts the body centres
    by the same offsets (periodic wrap and minimum-image lever arms)."""
    w = tiny_moving_body(second_body=True)
    w.params["e0"] = 0.5
    shift = (3, -4, 5)  # (z, y, x)
    o1 = _run(oracle_mod, w, 30)
    rho2 = np.roll(w.rho0, shift, axis=(0, 1, 2))
    phi2 = np.roll(w.phi0, shift, axis=(1, 2, 3))
    o2 = oracle_mod.Oracle(w.params, w.bodies, rho2, phi2)
    o2.step(30)
    assert np.max(np.abs(np.roll(o1.rho(), shift, axis=(0, 1, 2)) - o2.rho())) < 1e-12
    assert np.max(np.abs(np.roll(o1.phi(), shift, axis=(1, 2, 3)) - o2.phi())) < 1e-12
    b1, b2 = o1.bodies(), o2.bodies()
    assert np.allclose(b1["F"], b2["F"], atol=1e-12)
    assert np.allclose(b1["T"], b2["T"], atol=1e-11)
    n = np.array(w.shape[::-1], dtype=float)
    dX = (b2["X"] - b1["X"] - np.array(shift[::-1])) / n
    assert np.allclose(dX - np.round(dX), 0.0, atol=1e-12)


def test_repulsion_matches_brute_force_pair_sum(oracle_mod):
    """Solid-solid repulsion (Sec. 3.1.2) against an O(N^2) sum over every pair of solid nodes of
    two bodies: f = e0 (n / r_c) (x_i - x_j)/|x_i - x_j| |(|x_i - x_j| - r_c)/r_c|^(n-1) for
    |x_i - x_j| < r_c on the body at x_i; opposite on the other; torques about the centres."""
    shape = (12, 11, 16)
    nz, ny, nx = shape
    c1, c2 = (5.3, 5.2, 6.1), (10.4, 5.9, 5.7)
    phi = np.stack([sphere_phi(shape, c1, 2.6, 1.0), sphere_phi(shape, c2, 2.4, 1.0)])
    p = params(shape, 2, e0=0.7, kinetics=0, motion=0, G=0.0)
    o = oracle_mod.Oracle(p, [body(), body()], np.zeros(shape), phi)
    o.step(1)
    solid, owner = o.mask()
    X = o.bodies()["X"]
    pts = [np.argwhere((solid == 1) & (owner == b))[:, ::-1].astype(float) for b in (0, 1)]
    assert len(pts[0]) > 3 and len(pts[1]) > 3
    L = np.array([nx, ny, nz], float)
    F = np.zeros((2, 3))
    T = np.zeros((2, 3))
    rc, n, e0 = 3.0, 4.0, 0.7
    for pi in pts[0]:
        for qj in pts[1]:
            d = pi - qj
            d -= L * np.floor(d / L + 0.5)
            r = np.linalg.norm(d)
            if r >= rc:
                continue
            f = e0 * (n / rc) * d / r * abs((r - rc) / rc) ** (n - 1)
            F[0] += f
            F[1] -= f
            r1 = pi - X[0]
            r1 -= L * np.floor(r1 / L + 0.5)
            r2 = qj - X[1]
            r2 -= L * np.floor(r2 / L + 0.5)
            T[0] += np.cross(r1, f)
            T[1] -= np.cross(r2, f)
    rep = o.force_parts()["rep"]
    assert np.abs(F).max() > 1e-3
    assert np.allclose(rep, F, rtol=1e-12, atol=1e-14)
    b = o.bodies()
    assert np.allclose(b["T"], T, rtol=1e-12, atol=1e-13)  # empty fluid: torque is repulsion only
    # repulsive: body 0 (left) is pushed towards -x
    assert F[0, 0] < 0


def test_force_free_body_moves_uniformly(oracle_mod):
    """A body in an empty fluid feels no force: X_n = X_0 + n V, omega constant."""
    shape = (14, 13, 15)
    phi = sphere_phi(shape, (6.0, 6.5, 7.0), 3.0, 2.0)[None]
    V, Wv = (0.021, -0.013, 0.008), (0.001, -0.002, 0.003)
    p = params(shape, 1, kinetics=0, motion=1, G=-5.0)
    o = oracle_mod.Oracle(p, [body(v=V, w=Wv, fixed=0, mass_density=4.0)], np.zeros(shape), phi)
    X0 = o.bodies()["X"].copy()
    o.step(40)
    b = o.bodies()
    assert np.allclose(b["X"], X0 + 40 * np.array(V), atol=1e-12)
    assert np.allclose(b["W"], Wv, atol=1e-15)
    assert np.all(b["F"] == 0.0)


def test_body_kinematics_semi_implicit_euler(oracle_mod):
    """Rigid-body update (Sec. 3.1.1) is semi-implicit Euler with dt = 1: V += F/M, X += V,
    omega += I^-1 T, with F, T the forces the step reports."""
    w = tiny_moving_body(second_body=True)
    w.params["e0"] = 0.5
    o = oracle_mod.Oracle(w.params, w.bodies, w.rho0, w.phi0)
    c = o.body_consts()
    o.step(5)
    b0 = o.bodies()
    o.step(1)
    b1 = o.bodies()
    V = b0["V"] + b1["F"] / c["M"][:, None]
    assert np.allclose(b1["V"], V, rtol=1e-14, atol=1e-18)
    assert np.allclose(b1["X"], b0["X"] + V, rtol=1e-14, atol=1e-14)
    Wn = b0["W"] + np.einsum("bij,bj->bi", c["Iinv"], b1["T"])
    assert np.allclose(b1["W"], Wn, rtol=1e-13, atol=1e-18)


def test_inertia_of_uniform_ball(oracle_mod):
    """Mass, centre and inertia from the phase field at t = 0: for a sharp voxel ball the tensor
    equals the direct voxel sum rho_s sum (r^2 I - r r^T), diagonal by symmetry."""
    shape = (16, 16, 16)
    z, y, x = np.meshgrid(*(np.arange(16.0),) * 3, indexing="ij")
    ctr = np.array([7.0, 8.0, 7.5])
    ball = (((x - ctr[0]) ** 2 + (y - ctr[1]) ** 2 + (z - ctr[2]) ** 2) <= 4.2 ** 2).astype(float)
    p = params(shape, 1, kinetics=0, motion=0)
    o = oracle_mod.Oracle(p, [body(mass_density=2.5)], np.zeros(shape), ball[None])
    c = o.body_consts()
    X = o.bodies()["X"][0]
    assert np.allclose(X, ctr, atol=1e-12)
    assert abs(c["M"][0] - 2.5 * ball.sum()) < 1e-9
    r = np.stack([x - ctr[0], y - ctr[1], z - ctr[2]], -1)[ball > 0]
    I = 2.5 * ((r ** 2).sum(1).sum() * np.eye(3) - r.T @ r)
    assert np.allclose(np.linalg.inv(c["Iinv"][0]), I, rtol=1e-10)


def test_plate_solid_nodes_are_the_core():
    """Reading of the 16x16x2 plates: the solid nodes (fluid fraction < 0.05) are exactly the
    core cells; the faces are 8 cells apart."""
    w = plates_bridge()
    solid = (1.0 - w.phi0.sum(0)) < 0.05
    assert solid.sum() == 2 * 16 * 16 * 2
    zs = np.unique(np.argwhere(solid)[:, 0])
    assert list(zs) == [10, 11, 20, 21]
