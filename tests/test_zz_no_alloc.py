"""GPU: pf_lbm_step_noalloc (force partials in the library's static device array) against
pf_lbm_step (partials in the handle's workspace), through the C-ABI.

Both run the same kernels with the same arithmetic, so every output must agree bit for bit.  Two
calls in a row: first a 128^3 two-sphere bridge, whose force scan runs the largest grid (256
blocks) and fills the static array, then a smaller grid with moving, rotating bodies, node
conversions and repulsion (a few blocks), which must not see the first call's leftovers.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from parity_helpers import log  # noqa: E402


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available()
    return torch


def _same(a, b):
    for name in ("rho", "phi"):
        x, y = getattr(a, name)(), getattr(b, name)()
        assert np.array_equal(x, y), name
    ba, bb = a.bodies(), b.bodies()
    for k in ("F", "T", "X", "V", "W"):
        assert np.array_equal(ba[k], bb[k]), k
    assert a.diag() == b.diag()


def _pair(w, steps, precision):
    from paper_1902_10432_amd import binding as B
    from paper_1902_10432_amd.simulation import Simulation
    log(f"case {w.name} shape={w.shape} steps={steps} {precision}: pf_lbm_step vs pf_lbm_step_noalloc")
    ref = Simulation(w.params, w.bodies, w.rho0, w.phi0, precision=precision)
    ref.step(steps)
    sim = Simulation(w.params, w.bodies, w.rho0, w.phi0, precision=precision)
    done = 0
    for chunk in (1, steps // 2, steps - steps // 2 - 1):  # several calls, odd and even starts
        rc = B.pf_lbm_step_noalloc(sim._h, chunk)
        assert rc == B.PF_LBM_OK, B.pf_lbm_last_error(sim._h)
        done += chunk
    assert done == steps
    _same(sim, ref)
    return sim, ref


def test_noalloc_matches_step_large_then_small(torch_cuda):
    from pflbm_inputs import tiny_moving_body, two_spheres_bridge
    _pair(two_spheres_bridge(), 12, "fp32")
    w = tiny_moving_body(second_body=True)
    w.params["e0"] = 0.5
    sim, _ = _pair(w, 40, "fp64")
    assert sim.diag()["n_f2s"] > 0


def test_noalloc_rejects_timing_mode(torch_cuda):
    from paper_1902_10432_amd import binding as B
    from paper_1902_10432_amd.simulation import Simulation
    from pflbm_inputs import tiny_moving_body
    w = tiny_moving_body()
    sim = Simulation(w.params, w.bodies, w.rho0, w.phi0, precision="fp32")
    sim.timing(True)
    assert B.pf_lbm_step_noalloc(sim._h, 1) == B.PF_LBM_EINVAL
    sim.timing(False)
    assert B.pf_lbm_step_noalloc(sim._h, 2) == B.PF_LBM_OK
    assert B.pf_lbm_step_noalloc(sim._h, -1) == B.PF_LBM_EINVAL
