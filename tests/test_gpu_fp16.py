"""GPU: the FP16 population-storage form against the FP64 CPU oracle.

Populations are stored as FP16 deviations from w_i rho_ref with FP32 arithmetic; phase fields,
body sums and the rigid-body update stay FP64.  The bar is the body force within 1e-3, measured
as |dF| / max(|F_oracle|, pi sigma R) after the stated steps; density and phase fields are
reported and bounded by the FP16 resolution (an FP16 deviation of order 0.3 carries an absolute
rounding error of about 1e-4 per population and step).
"""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from parity_helpers import errors, log  # noqa: E402
from pflbm_inputs import plates_bridge, tiny_moving_body, two_spheres_bridge  # noqa: E402

SIGMA = 3.3e-2


_print = log


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available()
    return torch


def _run(oracle_mod, w, steps):
    from paper_1902_10432_amd.simulation import Simulation
    _print(f"case {w.name} shape={w.shape} steps={steps} fp16")
    sim = Simulation(w.params, w.bodies, w.rho0, w.phi0, precision="fp16")
    sim.step(steps)
    ref = oracle_mod.Oracle(w.params, w.bodies, w.rho0, w.phi0)
    ref.step(steps)
    return sim, ref


def _errors(sim, ref, steps, force_scale, lever):
    out = errors(sim, ref, steps, force_scale=force_scale, lever=lever)
    out["mass"] = abs(float(np.sum(sim.rho(), dtype=np.float64)) / float(np.sum(ref.rho())) - 1.0)
    _print(f"  mass={out['mass']:.3e}")
    return out


# every body quantity (force, torque, position, velocity, angular velocity) within the force bar
def _bodies_ok(e, tol=1e-3):
    return all(e[k] < tol for k in ("F", "T", "V", "X", "W"))


def test_fp16_plates_bridge_200_steps(oracle_mod, torch_cuda):
    w = plates_bridge()
    sim, ref = _run(oracle_mod, w, 200)
    e = _errors(sim, ref, 200, math.pi * SIGMA * 6.0, 8.0)
    assert _bodies_ok(e)
    assert e["rho"] < 2e-3 and e["phi"] < 1e-4 and e["mass"] < 1e-3
    assert e["mask_mismatch"] == 0


def test_fp16_moving_bodies_with_conversion(oracle_mod, torch_cuda):
    w = tiny_moving_body(second_body=True)
    w.params["e0"] = 0.5
    sim, ref = _run(oracle_mod, w, 60)
    e = _errors(sim, ref, 60, math.pi * SIGMA * 2.0, 3.0)
    assert _bodies_ok(e) and e["rho"] < 2e-3
    assert sim.diag()["n_f2s"] == ref.diag()["n_f2s"] > 0


def test_fp16_two_spheres_slice(oracle_mod, torch_cuda):
    w = two_spheres_bridge()
    sim, ref = _run(oracle_mod, w, 4)
    e = _errors(sim, ref, 4, math.pi * SIGMA * 20.0, 20.0)
    assert _bodies_ok(e) and e["rho"] < 2e-3 and e["mask_mismatch"] == 0
