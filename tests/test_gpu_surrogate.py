"""GPU: what the trained surrogate gains over the field method, end to end at reduced size.

The same pipeline as the full run (paper_1902_10432_amd.deploy), smaller: 32 sweep bridges in
boxes of 48^3..96^3 solved for 1200 steps (force over the last 600), GPU training of the 4 x 128
network with the library's kernels, then a 1000-sphere run (3 % liquid, radii 12..18) for 200
steps with 8 bridges re-solved at 96^3 under the same protocol every 100 steps, the judged bridges
refining the network after each judgement.  Checks:
* training lowers the loss;
* a network bridge force costs at least 10^4 times less GPU time than a field solve of the bridge
  (measured gain is about 2 x 10^6);
* the network's error on the judged bridges is below the RMS of their field forces (it does better
  than no bridge force at all), and every bridge it misses by more than the tolerance runs on the
  field force afterwards (fallback);
* the refinement changes the network, and the run stays finite.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _print(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available()
    return torch


def test_surrogate_gain_over_field_solves(torch_cuda):
    from paper_1902_10432_amd import deploy as Dp
    _print("case surrogate pipeline: sweep 32 x 1200 steps, train, 1000 spheres x 200 steps, judge 8 twice")
    X, y, _ = Dp.training_set(32, seeds=(0,), steps=1200, window=600, log=_print, max_len=96)
    norm = Dp.normalisation(X, y)
    net, rep = Dp.train(X, y, norm, log=_print)
    assert rep["loss_final"] < rep["loss_first"]
    p0 = net.params()
    s = Dp.deploy(net, norm, n=1000, steps=200, judge_every=100, judge_pairs=8, judge_steps=1200, judge_window=600,
                  train_data=(X, y), refine_steps=20, log=_print)
    r = s["rounds"][-1]
    assert not np.array_equal(net.params(), p0)
    assert len(s["rounds"]) == 2 and all(q["refine_s"] > 0 for q in s["rounds"])
    _print(f"  speedup per bridge {s['speedup_per_bridge']:.3g}, RMSE {s['rmse']:.3e} vs field RMS {s['rms_field']:.3e}")
    assert s["speedup_per_bridge"] > 1e4
    assert r["x_finite"] and r["judged"] == 8 and r["bridges"] > 500
    assert s["rmse"] < s["rms_field"]
