"""GPU: the many-sphere rigid-body run with surrogate bridge forces against the FP64 run oracle.

* bridge list bit-exact (integer work); bridge features to round-off;
* bridge forces against the FP64 network oracle with BF16 operand rounding (the GPU network's
  arithmetic), bound 2e-3 of the RMS force (as for the network alone);
* per-sphere force sums and one semi-implicit Euler step against the oracle given the GPU's own
  bridge forces, to round-off;
* overrides replace exactly the listed pairs;
* 20 steps against the oracle run with the oracle network: position differences within 1e-2 of
  the distance moved (the two networks differ by FP32 accumulation order, amplified by contacts);
* capacity overflow is reported (ENOMEM) and leaves the state unchanged.
Cases: 300 spheres (one thread-chunk per sphere in the row scan) and 1500 (two per thread), both
with overlapping spheres so the contact law is exercised.
"""
import math
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from oracle import dem_oracle as D  # noqa: E402
from oracle import mlp_oracle as M  # noqa: E402

NORM = {"in_shift": [0.2, 0.8, 0.5, 0.5], "in_scale": [3.0, 5.0, 2.0, 2.0], "out_shift": 0.5, "out_scale": 0.3}
KN, GN, DT, RHO, THETA, CFRAC, GMIN, GMAX = 4.0, 0.5, 0.2, 1.0, 0.5, 0.05, 0.25, 1.5


def _print(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available()
    return torch


def _net(seed=5):
    from paper_1902_10432_amd.surrogate import Surrogate
    net = Surrogate(4, 64, 2, max_batch=8192, seed=seed)
    rng = np.random.default_rng(seed)
    p = M.to_bf16(net.params()).astype(np.float32)
    k = 0
    for o, i in M.layer_shapes(4, 64, 2):
        k += o * i
        p[k:k + o] = rng.normal(0.0, 0.2, o).astype(np.float32)
        k += o
    net.set_params(p)
    return net, p.astype(np.float64)


def _spheres(n, seed):
    rng = np.random.default_rng(seed)
    L = (n * 4.0 / 3.0 * math.pi * 2.5 ** 3 / 0.3) ** (1.0 / 3.0)
    R = rng.uniform(2.0, 3.0, n)
    x = rng.uniform(0.0, L, (n, 3))
    v = rng.normal(0.0, 0.01, (n, 3))
    return L, R, x, v


def _run(net, n, L, R, x, v, cap=32):
    from paper_1902_10432_amd.surrogate import SphereRun, dem_config
    cfg = dem_config(n, L, DT, RHO, KN, GN, THETA, CFRAC, GMIN, GMAX, NORM, max_neighbours=cap, max_pairs=8192)
    return SphereRun(net, cfg, R, x, v)


def _oracle_bridge_forces(p, R, ij, gaps):
    f, rs = D.features(R[ij[:, 0]], R[ij[:, 1]], gaps, THETA, CFRAC, GMIN)
    X = ((f - np.array(NORM["in_shift"], dtype=np.float32).astype(np.float64))
         * np.array(NORM["in_scale"], dtype=np.float32).astype(np.float64)).astype(np.float32)
    y, _, _ = M.forward(p, X, 4, 64, 2, bf16_acts=True)
    return (y * np.float64(np.float32(NORM["out_scale"])) + np.float64(np.float32(NORM["out_shift"]))) * rs, f


@pytest.mark.parametrize("n", [300, 1500])
def test_evaluate_and_one_step_against_oracle(torch_cuda, n):
    _print(f"case evaluate n={n}")
    net, p = _net()
    L, R, x, v = _spheres(n, seed=n)
    run = _run(net, n, L, R, x, v)
    run.evaluate()
    got = run.pairs()
    ij, gaps, units = D.bridges(x, R, L, GMAX)
    _print(f"  {len(ij)} bridges, {int((gaps < 0).sum())} contacts")
    assert len(ij) > n // 4 and (gaps < 0).sum() > 5
    assert np.array_equal(got["ij"], ij)
    fb_ref, feat = _oracle_bridge_forces(p, R, ij, gaps)
    assert np.abs(got["features"] - feat).max() <= 1e-13 * np.abs(feat).max()
    rms = math.sqrt(float((fb_ref ** 2).mean()))
    err = np.abs(got["force"] - fb_ref).max() / rms
    _print(f"  bridge force max err / rms {err:.2e}")
    assert err <= 2e-3
    st = run.state()
    F_ref = D.forces(x, v, R, L, ij, units, gaps, got["force"], KN, GN)
    assert np.abs(st["F"] - F_ref).max() <= 1e-12 * np.abs(F_ref).max()
    run.step(1)
    st1 = run.state()
    x1, v1 = D.integrate(x, v, st["F"], R, RHO, DT, L)
    assert np.abs(st1["v"] - v1).max() <= 1e-13 * np.abs(v1).max()
    dx = D.min_image(st1["x"] - x1, L)
    assert np.abs(dx).max() <= 1e-12 * L


def test_overrides_replace_listed_pairs(torch_cuda):
    net, _ = _net()
    n = 300
    L, R, x, v = _spheres(n, seed=7)
    run = _run(net, n, L, R, x, v)
    run.evaluate()
    base = run.pairs()
    sel = [0, 5, len(base["ij"]) - 1]
    ov = np.array([1.25, -0.5, 3.0])
    run.set_overrides(base["ij"][sel][:, ::-1], ov)   # either order
    run.evaluate()
    got = run.pairs()
    assert np.array_equal(got["ij"], base["ij"])
    assert np.array_equal(got["force"][sel], ov)
    keep = np.setdiff1d(np.arange(len(base["ij"])), sel)
    assert np.array_equal(got["force"][keep], base["force"][keep])
    run.set_overrides(np.zeros((0, 2)), np.zeros(0))
    run.evaluate()
    assert np.array_equal(run.pairs()["force"], base["force"])


def test_twenty_steps_against_oracle_run(torch_cuda):
    net, p = _net()
    n = 300
    L, R, x, v = _spheres(n, seed=11)
    run = _run(net, n, L, R, x, v)
    run.step(20)
    xo, vo = x.copy(), v.copy()
    for _ in range(20):
        xo, vo, _ = D.step(xo, vo, R, L, DT, RHO, KN, GN, GMAX,
                           lambda ij, g: _oracle_bridge_forces(p, R, ij, g)[0])
    st = run.state()
    d = np.abs(D.min_image(st["x"] - xo, L)).max()
    moved = np.abs(D.min_image(xo - x, L)).max()
    _print(f"  20 steps: max |dx| {d:.2e} (max displacement {moved:.2e})")
    assert moved > 1e-2 and d <= 1e-2 * moved


def test_capacity_overflow_reported(torch_cuda):
    from paper_1902_10432_amd.surrogate import SurrogateError
    net, _ = _net()
    n = 300
    L, R, x, v = _spheres(n, seed=3)
    run = _run(net, n, L, R, x, v, cap=1)
    with pytest.raises(SurrogateError, match="max_neighbours"):
        run.step(1)
    st = run.state()
    assert np.array_equal(st["x"], x) and np.array_equal(st["v"], v)
