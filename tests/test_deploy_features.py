"""Host-side checks of the surrogate pipeline: the features of the training bridges
(deploy.features, from the radii, gap, placed liquid volume and angle) are the features the
many-sphere run computes for a bridge (the run oracle's definition, which the GPU run matches),
and the normalisation maps the training set to zero mean and unit spread."""
import math

import numpy as np

from oracle import dem_oracle as D


def test_training_features_match_the_run_features():
    from paper_1902_10432_amd import deploy as Dp
    rng = np.random.default_rng(0)
    r1, r2 = rng.uniform(8, 30, 50), rng.uniform(8, 30, 50)
    gap = rng.uniform(-1.0, 8.0, 50)
    c, theta = 0.07, math.radians(35.0)
    v_l = c / (1 - c) * 4.0 / 3.0 * math.pi * (r1 ** 3 + r2 ** 3)
    f_train, rs_train = Dp.features(r1, r2, gap, v_l, theta)
    f_run, rs_run = D.features(r1, r2, gap, theta, c, Dp.GAP_MIN)
    assert np.allclose(f_train, f_run, rtol=1e-14, atol=0)
    assert np.allclose(rs_train, rs_run, rtol=1e-15, atol=0)


def test_normalisation_standardises():
    from paper_1902_10432_amd import deploy as Dp
    rng = np.random.default_rng(1)
    X = rng.normal([0.3, 0.7, 1.5, 0.5], [0.1, 0.2, 0.8, 0.3], (200, 4))
    X[:, 3] = 0.5  # a constant feature keeps scale 1
    y = rng.normal(0.05, 0.02, 200)
    n = Dp.normalisation(X, y)
    Z = (X - np.array(n["in_shift"])) * np.array(n["in_scale"])
    assert np.allclose(Z[:, :3].mean(0), 0, atol=1e-12) and np.allclose(Z[:, :3].std(0), 1, atol=1e-12)
    assert n["in_scale"][3] == 1.0
    assert abs(((y - n["out_shift"]) / n["out_scale"]).std() - 1) < 1e-12
