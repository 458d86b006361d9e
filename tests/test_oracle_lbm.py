"""Pins of the oracle's fluid part against textbook lattice-Boltzmann facts and exact special
cases (Sec. 3.2.1 collision, equilibrium, Guo forcing; Sec. 3.2.2 half-way bounce-back).

Every expectation here is fixed by mathematics outside the oracle: lattice moment identities,
exact steady states of the discrete scheme, conservation laws."""
import itertools
import math

import numpy as np
import pytest

from oracle_helpers import body, params, slab_phi
from pflbm_inputs import uniform_fluid


LATTICES = [19, 27]


@pytest.mark.parametrize("lattice", LATTICES)
def test_lattice_moment_identities(oracle_mod, lattice):
    w = uniform_fluid((2, 2, 2), lattice=lattice)
    o = oracle_mod.Oracle(w.params, w.bodies, w.rho0, w.phi0)
    c, wt = o.lattice()
    assert len({tuple(v) for v in c}) == lattice
    assert all((v ** 2).sum() <= (3 if lattice == 27 else 2) for v in c)
    # sixth moment along the body diagonal tells the two sets apart: D3Q27's weights are the
    # tensor product of the 1-D weights (2/3, 1/6, 1/6), so sum w cx^2 cy^2 cz^2 = (1/3)^3
    assert abs((wt * c[:, 0] ** 2 * c[:, 1] ** 2 * c[:, 2] ** 2).sum() - (1 / 27 if lattice == 27 else 0)) < 1e-15
    assert abs(wt.sum() - 1.0) < 1e-15
    assert np.allclose((wt[:, None] * c).sum(0), 0.0, atol=1e-16)
    I = np.eye(3)
    for a, b in itertools.product(range(3), repeat=2):
        assert abs((wt * c[:, a] * c[:, b]).sum() - I[a, b] / 3.0) < 1e-15
    # isotropic fourth moment: (d_ab d_cd + d_ac d_bd + d_ad d_bc) / 9
    for a, b, cc, d in itertools.product(range(3), repeat=4):
        want = (I[a, b] * I[cc, d] + I[a, cc] * I[b, d] + I[a, d] * I[b, cc]) / 9.0
        assert abs((wt * c[:, a] * c[:, b] * c[:, cc] * c[:, d]).sum() - want) < 1e-15


@pytest.mark.parametrize("lattice", LATTICES)
@pytest.mark.parametrize("u", [(0.0, 0.0, 0.0), (0.05, -0.02, 0.01), (-0.1, 0.07, 0.03)])
def test_equilibrium_moments(oracle_mod, u, lattice):
    """The second-order equilibrium reproduces rho, rho u and rho (c_s^2 I + u u) exactly."""
    w = uniform_fluid((2, 2, 2), lattice=lattice)
    o = oracle_mod.Oracle(w.params, w.bodies, w.rho0, w.phi0)
    c, _ = o.lattice()
    rho = 1.3
    u = np.array(u)
    feq = o.equilibrium(rho, u)
    assert abs(feq.sum() - rho) < 1e-14
    assert np.allclose((feq[:, None] * c).sum(0), rho * u, atol=1e-15)
    P = np.einsum("i,ia,ib->ab", feq, c, c)
    assert np.allclose(P, rho * (np.eye(3) / 3.0 + np.outer(u, u)), atol=1e-14)


def test_rest_state_is_invariant(oracle_mod):
    """A uniform fluid at rest is a fixed point of the step for any coupling G."""
    w = uniform_fluid((6, 5, 7), rho=0.8, G=-5.0)
    o = oracle_mod.Oracle(w.params, w.bodies, w.rho0, w.phi0)
    f0 = o.populations().copy()
    o.step(10)
    assert np.max(np.abs(o.populations() - f0)) < 1e-15


def test_guo_uniform_force_momentum(oracle_mod):
    """A uniform force density F adds exactly F of momentum per node and step, and the physical
    momentum rho v = sum c f + F/2 after n steps equals (n + 1/2) F (Guo forcing, Sec. 3.2.1)."""
    F = np.array([1e-5, -2e-5, 3e-5])
    w = uniform_fluid((4, 3, 5), rho=1.0, G=0.0, fext=tuple(F))
    o = oracle_mod.Oracle(w.params, w.bodies, w.rho0, w.phi0)
    n = 25
    o.step(n)
    j = o.mom().reshape(3, -1)
    assert np.allclose(j, (n * F)[:, None], rtol=0, atol=1e-16 * n + 1e-18)
    assert np.allclose(o.rho(), 1.0, atol=1e-14)


@pytest.mark.parametrize("lattice,tau", [(19, 0.8), (27, 1.1)])
def test_shear_wave_decay_rate(oracle_mod, lattice, tau):
    """With G = 0 a transverse shear wave decays at nu k^2, nu = c_s^2 (tau - 1/2) (BGK viscosity);
    the lattice correction is O(k^2) relative, far below the 1 % tolerance at k = 2 pi / 64."""
    L, U = 64, 1e-3
    shape = (1, L, 1)
    w = uniform_fluid(shape, rho=1.0, G=0.0, tau=tau, lattice=lattice)
    o = oracle_mod.Oracle(w.params, w.bodies, w.rho0, w.phi0)
    y = np.arange(L)
    k = 2 * math.pi / L
    f = np.stack([o.equilibrium(1.0, (U * math.sin(k * yy), 0.0, 0.0)) for yy in y]).reshape(1, L, 1, lattice)
    o.set_populations(f)

    def amp():
        jx = o.mom()[0, 0, :, 0]
        return 2.0 / L * (jx * np.sin(k * y)).sum()

    o.step(50)
    a1 = amp()
    o.step(400)
    a2 = amp()
    rate = -math.log(a2 / a1) / 400
    nu = (tau - 0.5) / 3.0
    assert abs(rate / (nu * k * k) - 1.0) < 1e-2


@pytest.mark.parametrize("lattice", LATTICES)
def test_poiseuille_exact_at_magic_tau(oracle_mod, lattice):
    """Body-force-driven channel flow between half-way bounce-back walls: the BGK steady state is
    the exact parabola u(z) = g (z - z0)(z1 - z) / (2 nu rho) with walls half-way between the
    solid and fluid nodes when (tau - 1/2)^2 = 3/16."""
    H = 9
    shape = (H + 1, 1, 2)
    tau = 0.5 + math.sqrt(3.0 / 16.0)
    g = 1e-6
    p = params(shape, 1, tau=tau, G=0.0, fext=(g, 0.0, 0.0), kinetics=0, motion=0, repulsion=0, lattice=lattice)
    phi = slab_phi(shape, [0])[None]
    o = oracle_mod.Oracle(p, [body()], np.ones(shape), phi)
    o.step(6000)
    rho = o.rho()[:, 0, 0]
    ux = (o.mom()[0, :, 0, 0] + 0.5 * g) / np.where(rho > 0, rho, 1)
    nu = (tau - 0.5) / 3.0
    z = np.arange(1, H + 1)
    want = g * (z - 0.5) * (H + 0.5 - z) / (2 * nu * 1.0)
    assert np.max(np.abs(ux[1:] - want)) < 1e-9 * want.max()
    assert abs(rho[0]) == 0.0


@pytest.mark.parametrize("lattice", LATTICES)
def test_couette_linear_profile_moving_wall(oracle_mod, lattice):
    """Two walls, one moving tangentially with U: the steady state is the exact linear profile
    from U to 0 between the half-way wall positions (moving-wall bounce-back, Sec. 3.2.2)."""
    H = 7
    nz = 2 * H + 2
    shape = (nz, 1, 3)
    U = 1e-3
    p = params(shape, 2, tau=1.0, G=0.0, kinetics=0, motion=0, repulsion=0, lattice=lattice)
    phi = np.stack([slab_phi(shape, [0]), slab_phi(shape, [H + 1])])
    o = oracle_mod.Oracle(p, [body(v=(U, 0, 0)), body()], np.ones(shape), phi)
    o.step(6000)
    rho = o.rho()[:, 0, 0]
    ux = o.mom()[0, :, 0, 0] / np.where(rho > 0, rho, 1)
    z = np.arange(1, H + 1)
    want = U * (H + 0.5 - z) / H
    assert np.max(np.abs(ux[1:H + 1] - want)) < 1e-10
    # the second channel (from the resting wall back to the moving one through the boundary)
    want2 = U * (z - 0.5) / H
    assert np.max(np.abs(ux[H + 2:] - want2)) < 1e-10
    # tangential wall motion brings no net mass: the rest-population correction sums to zero
    assert abs(rho[1:H + 1].mean() - 1.0) < 1e-12
