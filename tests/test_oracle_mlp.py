"""Pins of the FP64 surrogate-network oracle: the backward pass against central finite
differences of the loss, the forward pass against a hand-built single-unit network, and the BF16
rounding against its definition (round to nearest, ties to even, of the FP32 value)."""
import numpy as np

from oracle import mlp_oracle as M


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(3)
    n_in, hidden, layers = 4, 16, 3
    n_par = sum(o * i + o for o, i in M.layer_shapes(n_in, hidden, layers))
    p = rng.normal(0.0, 0.4, n_par)
    x = rng.normal(0.0, 1.0, (7, n_in))
    t = rng.normal(0.0, 1.0, 7)
    _, g = M.loss_and_grad(p, x, t, n_in, hidden, layers)
    h = 1e-6
    for k in rng.choice(n_par, 60, replace=False):
        e = np.zeros(n_par)
        e[k] = h
        fd = (M.loss_and_grad(p + e, x, t, n_in, hidden, layers)[0]
              - M.loss_and_grad(p - e, x, t, n_in, hidden, layers)[0]) / (2 * h)
        assert abs(fd - g[k]) <= 1e-7 * max(1.0, abs(fd))


def test_forward_of_a_single_unit_network():
    # one input, hidden width 1, one hidden layer: y = w1 silu(w0 x + b0) + b1
    w0, b0, w1, b1 = 0.7, -0.2, 1.3, 0.05
    p = np.array([w0, b0, w1, b1])
    x = np.array([[0.5], [-1.5], [2.0]])
    y, _, _ = M.forward(p, x, 1, 1, 1)
    z = w0 * x[:, 0] + b0
    assert np.allclose(y, w1 * z / (1 + np.exp(-z)) + b1, rtol=0, atol=1e-15)


def test_bf16_rounding():
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 2 ** -9, 1.0 + 3 * 2 ** -9, -3.14159, 1e-3], dtype=np.float32)
    r = M.to_bf16(vals)
    # 8 significant bits: 1 + 2^-8 is not representable; 1 + 2^-9 ties to even -> 1
    assert r[0] == 1.0 and r[2] == 1.0
    assert r[1] == 1.0 or r[1] == 1.0 + 2 ** -7
    assert r[3] == 1.0 + 2 ** -7              # 1.0117 rounds up to 1 + 2^-7
    assert abs(r[4] - (-3.140625)) < 1e-12    # nearest BF16 of pi
    assert abs(r[5] / 1e-3 - 1) < 2 ** -8


def test_bf16_activation_rounding_only_touches_operands():
    # every operand that enters a product is BF16-exact, and the rounding moves a generic
    # output by a small relative amount (each rounding is at most 2^-9 relative)
    rng = np.random.default_rng(5)
    n_in, hidden, layers = 4, 16, 2
    n_par = sum(o * i + o for o, i in M.layer_shapes(n_in, hidden, layers))
    p = rng.normal(0.0, 0.5, n_par)
    x = rng.normal(0.0, 1.0, (50, n_in))
    y, _, _ = M.forward(p, x, n_in, hidden, layers)
    yb, _, acts = M.forward(p, x, n_in, hidden, layers, bf16_acts=True)
    for a in acts[:-1]:
        assert np.array_equal(a, M.to_bf16(a))
    d = np.linalg.norm(y - yb) / np.linalg.norm(y)
    assert 1e-5 < d < 2e-2
