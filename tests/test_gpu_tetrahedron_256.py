"""GPU parity at the size of the benchmark: the 256^3 four-sphere workload (spheres R = 24 at the
vertices of a regular tetrahedron, central drop of 5 %, seeded 1e-3 perturbations of the phase
fields, the paper's tau = 1.1) against the FP64 oracle, element by element after a 4-step slice
(the oracle takes a few CPU seconds per step at this size).

This is the launch configuration the benchmark times (the fluid pass over the whole 256^3 grid,
four bodies, the phase-field kernels on the active tiles of the box).  Bars (parity_helpers documents how each figure is measured):
  FP64         fields <= 1e-11 (relative L2), 1e-10 per node; body quantities <= 1e-9
  FP32         fields <= 1e-5, 1e-4 per node; body quantities <= 1e-4
  FP16 storage body quantities <= 1e-3 (force over max(|F_oracle|, pi sigma R)); density
               <= 2e-3 (relative L2) and 5e-3 per node (FP16 keeps 11 significant bits of each
               stored deviation); phase fields (FP64 in every form) <= 1e-5.
"""
import math

import numpy as np
import pytest

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]

from parity_helpers import check, errors, log, snapshot  # noqa: E402

SIGMA = 3.3e-2
STEPS = 4
RADIUS = 24.0

BARS = {
    "fp64": dict(tol_field=1e-11, tol_force=1e-9, tol_node=1e-10),
    "fp32": dict(tol_field=1e-5, tol_force=1e-4, tol_node=1e-4),
    "fp16": dict(tol_field=2e-3, tol_force=1e-3, tol_node=5e-3, tol_phi=1e-5, tol_mom=2e-3),
}


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available()
    return torch


@pytest.fixture(scope="module")
def tetrahedron(oracle_mod):
    from pflbm_inputs import tetrahedron_drop
    log("case tetrahedron_drop 256^3 tau 1.1: generating inputs")
    w = tetrahedron_drop(tau=1.1)
    log(f"  oracle: {STEPS} steps")
    ref = oracle_mod.Oracle(w.params, w.bodies, w.rho0, w.phi0)
    ref.step(STEPS)
    snap = snapshot(ref)
    snap["diag"] = ref.diag()
    del ref
    return w, snap


@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp16"])
def test_tetrahedron_256_slice(tetrahedron, torch_cuda, precision):
    from paper_1902_10432_amd.simulation import Simulation
    w, snap = tetrahedron
    log(f"case tetrahedron_drop 256^3 tau 1.1 steps={STEPS} {precision}")
    sim = Simulation(w.params, w.bodies, w.rho0, w.phi0, precision=precision)
    sim.step(STEPS)
    out = errors(sim, None, STEPS, force_scale=math.pi * SIGMA * RADIUS, lever=RADIUS, ref_fields=snap)
    d = sim.diag()
    assert d["n_f2s"] == snap["diag"]["n_f2s"] and d["n_s2f"] == snap["diag"]["n_s2f"]
    sim.close()
    del sim
    torch_cuda.cuda.empty_cache()
    check(out, **BARS[precision])
