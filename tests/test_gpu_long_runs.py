"""GPU: the full-length runs of the two large configurations, FP32 and FP16 storage against the
FP64 build (which matches the FP64 oracle at round-off on every short slice tested; a CPU oracle
run of these lengths would take hours).

* 128^3 two spheres (R = 20, gap 4, 2 % bridge, 30 degrees), FP32, 10,000 steps, motion on;
* 256^3 four spheres at the tetrahedron vertices (R = 24, 5 % central drop, seeded 1e-3
  perturbations), 5,000 steps, FP32 and FP16 storage, at the paper's tau = 1.1 (at tau = 1.0 the
  FP32 trajectory of this case turns unstable near step 900: the bodies' moving surfaces convert
  about ten nodes each way per step, every node that turns fluid starts empty as the method
  prescribes, and partly refilled nodes reach speeds above 0.6; the FP64 trajectory survives).
The runs are long enough for round-off to change the trajectory in detail (conversions and
pressure waves make the instantaneous force fluctuate), so the checks are on the body positions,
the fields and the force averaged over the last 1,000 steps.
"""
import math
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

SIGMA = 3.3e-2


def _print(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available()
    return torch


def _run(w, prec, steps, window=1000):
    from paper_1902_10432_amd.simulation import Simulation
    s = Simulation(w.params, w.bodies, w.rho0, w.phi0, precision=prec)
    done = 0
    while done < steps:
        k = min(1000, steps - done)
        s.step(k)
        done += k
        _print(f"  {prec} step {done}")
    h = s.force_history(window)
    out = {"Fmean": h[:, :, :3].mean(axis=0), "X": s.bodies()["X"], "rho": s.rho(), "phi": s.phi()}
    del s
    return out


def _diff(a, ref, scale):
    return {"F": float(np.abs(a["Fmean"] - ref["Fmean"]).max() / scale),
            "X": float(np.abs(a["X"] - ref["X"]).max()),
            "rho": float(np.linalg.norm(a["rho"] - ref["rho"]) / np.linalg.norm(ref["rho"])),
            "phi": float(np.linalg.norm(a["phi"] - ref["phi"]) / np.linalg.norm(ref["phi"]))}


def test_two_spheres_10000_steps_fp32(torch_cuda):
    from pflbm_inputs import two_spheres_bridge
    w = two_spheres_bridge()
    _print("case two_spheres_bridge 128^3 10000 steps fp64 / fp32")
    r64 = _run(w, "fp64", 10000)
    r32 = _run(w, "fp32", 10000)
    d = _diff(r32, r64, math.pi * SIGMA * 20.0)
    _print(f"  fp32 vs fp64: {d}")
    # measured: F 2.6e-4, X 1.1e-3 cells, rho 1.2e-3, phi 1.0e-4
    assert d["X"] < 5e-3 and d["rho"] < 5e-3 and d["phi"] < 5e-4 and d["F"] < 2e-3


def test_tetrahedron_5000_steps_fp32_fp16(torch_cuda):
    from pflbm_inputs import tetrahedron_drop
    w = tetrahedron_drop(tau=1.1)
    _print("case tetrahedron_drop 256^3 5000 steps tau 1.1 fp64 / fp32 / fp16")
    r64 = _run(w, "fp64", 5000)
    scale = math.pi * SIGMA * 24.0
    d32 = _diff(_run(w, "fp32", 5000), r64, scale)
    _print(f"  fp32 vs fp64: {d32}")
    d16 = _diff(_run(w, "fp16", 5000), r64, scale)
    _print(f"  fp16 vs fp64: {d16}")
    # measured: F 7.2e-3 (FP32) and 1.0e-2 (FP16) of pi sigma R, X 0.02 cells, rho 2.4-2.7 %,
    # phi 1.6-1.9e-3: FP16 storage stays as close to the FP64 trajectory as plain FP32
    for d in (d32, d16):
        assert d["X"] < 0.05 and d["rho"] < 0.05 and d["phi"] < 5e-3 and d["F"] < 0.03
    assert d16["F"] < 3 * max(d32["F"], 1e-3)
