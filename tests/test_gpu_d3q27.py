"""GPU parity on the D3Q27 lattice of Sec. 3.2.1 (the library against the FP64 oracle run on the
same lattice), at the paper's relaxation time tau = 1.1 where the workload allows.

Bounds as for D3Q19: FP64 at round-off (relative L2 <= 1e-11, body quantities <= 1e-9); FP32
relative L2 <= 1e-5 on density and phase fields and <= 1e-4 on body quantities after 200 steps
(force error over max(|F_oracle|, pi sigma R)); FP16 population storage <= 1e-3 on body
quantities."""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from pflbm_inputs import plates_bridge, tiny_moving_body, uniform_fluid  # noqa: E402
from parity_helpers import compare  # noqa: E402
from test_gpu_parity import FP32, FP64, SIGMA, _pair  # noqa: E402


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available()
    return torch


def test_d3q27_tiny_moving_bodies_fp64(oracle_mod, torch_cuda):
    w = tiny_moving_body(second_body=True, lattice=27, tau=1.1)
    w.params["e0"] = 0.5
    sim, ref = _pair(oracle_mod, w, 60, "fp64")
    compare(sim, ref, 60, lever=3.0, **FP64)
    dg, do = sim.diag(), ref.diag()
    assert dg["n_f2s"] == do["n_f2s"] and dg["n_s2f"] == do["n_s2f"] and dg["n_f2s"] > 0


@pytest.mark.parametrize("shape", [(7, 9, 13), (12, 1, 17)])
def test_d3q27_ragged_and_flat_grids_fp64(oracle_mod, torch_cuda, shape):
    from pflbm_inputs import coexistence_densities, liquid_density
    from pflbm_inputs.geometry import grid, mimg
    rv, rl = coexistence_densities()
    x, y, z = grid(shape)
    nz, ny, nx = shape
    d = np.sqrt(mimg(x - nx / 2, nx) ** 2 + mimg(y - ny / 2, ny) ** 2 + mimg(z - nz / 2, nz) ** 2) - min(nx, 6) / 2.5
    w = uniform_fluid(shape, G=-5.0, lattice=27, tau=1.1)
    w.rho0 = liquid_density(d, rl, rv, 3.0)
    sim, ref = _pair(oracle_mod, w, 30, "fp64")
    compare(sim, ref, 30, **FP64)


def test_d3q27_plates_bridge_fp64_200_steps(oracle_mod, torch_cuda):
    w = plates_bridge(lattice=27, tau=1.1)
    sim, ref = _pair(oracle_mod, w, 200, "fp64")
    compare(sim, ref, 200, lever=8.0, **FP64)


@pytest.mark.parametrize("precision,bars", [("fp32", FP32), ("fp16", dict(tol_field=1e-3, tol_force=1e-3, tol_node=2e-2))])
def test_d3q27_plates_bridge_reduced_precision(oracle_mod, torch_cuda, precision, bars):
    w = plates_bridge(lattice=27, tau=1.1)
    sim, ref = _pair(oracle_mod, w, 200, precision)
    compare(sim, ref, 200, force_scale=math.pi * SIGMA * 6.0, lever=8.0, **bars)


def test_d3q27_rest_state_and_mass(oracle_mod, torch_cuda):
    w = uniform_fluid((6, 5, 7), rho=0.8, G=-5.0, lattice=27)
    sim, ref = _pair(oracle_mod, w, 20, "fp32")
    assert np.abs(sim.rho() - 0.8).max() < 1e-6
    assert np.abs(sim.mom()).max() < 1e-7


def test_d3q27_fp16_moving_bodies_with_conversion(oracle_mod, torch_cuda):
    """FP16 population storage on D3Q27 through moving walls and node conversions (60 steps):
    body force within 1e-3 of max(|F|, pi sigma R), same conversion counts as the oracle."""
    w = tiny_moving_body(second_body=True, lattice=27, tau=1.1)
    w.params["e0"] = 0.5
    sim, ref = _pair(oracle_mod, w, 60, "fp16")
    out = compare(sim, ref, 60, tol_field=2e-3, tol_force=1e-3, tol_node=2e-2, force_scale=math.pi * SIGMA * 2.0,
                  lever=3.0)
    assert out["F"] < 1e-3
    assert sim.diag()["n_f2s"] == ref.diag()["n_f2s"] > 0


def test_d3q27_batch_matches_individual_runs(torch_cuda):
    from paper_1902_10432_amd.simulation import Simulation, step_batch
    from pflbm_inputs import bridge_pair
    args = [((24, 28, 40), 5.0, 6.5, 3.0, 0.05, 30.0), ((20, 26, 36), 4.5, 5.0, 2.5, 0.10, 10.0)]
    ws = [bridge_pair(*a, lattice=27) for a in args]
    alone = [Simulation(w.params, w.bodies, w.rho0, w.phi0, precision="fp32") for w in ws]
    for s in alone:
        s.step(21)
    together = [Simulation(w.params, w.bodies, w.rho0, w.phi0, precision="fp32") for w in ws]
    step_batch(together, 21)
    for a, b in zip(alone, together):
        assert np.array_equal(a.rho(), b.rho()) and np.array_equal(a.phi(), b.phi())
        assert np.array_equal(a.bodies()["F"], b.bodies()["F"])
