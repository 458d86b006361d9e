"""GPU: the surrogate network's BF16-MFMA forward and backward kernels against the FP64 network
oracle, and its Adam training.

Weights are set to BF16-exact values (so the kernels' BF16 weight copies hold them exactly) with
FP32 biases.  Two references per check:
* the oracle with BF16 operand rounding (inputs and hidden activations rounded to BF16 before
  each product): the kernels then differ only by FP32 accumulation order and, for gradients, the
  BF16 rounding of the back-propagated error; bounds 2e-3 (forward) and 1.5e-2 (gradients) relative;
* the plain FP64 oracle: bounds 3e-2 and 6e-2 relative (a BF16 operand carries 2^-9 relative
  rounding, through up to nine products).
Shapes cover K tails (n_in 3, 4, 16 < 32; hidden 48 = 32 + 16), M tails (batches 1, 37, 513,
1000) and a single hidden layer.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from oracle import mlp_oracle as M  # noqa: E402

CASES = [(4, 128, 4, 1000), (4, 48, 2, 37), (3, 16, 1, 1), (16, 64, 3, 513)]


def _print(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available()
    return torch


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300))


def _setup(torch, n_in, hidden, layers, n, seed):
    from paper_1902_10432_amd.surrogate import Surrogate
    net = Surrogate(n_in, hidden, layers, max_batch=max(n, 64), seed=seed)
    rng = np.random.default_rng(seed)
    p = M.to_bf16(net.params()).astype(np.float32)
    k = 0
    for o, i in M.layer_shapes(n_in, hidden, layers):
        k += o * i
        p[k:k + o] = rng.normal(0.0, 0.2, o).astype(np.float32)
        k += o
    net.set_params(p)
    x = rng.normal(0.0, 1.0, (n, n_in)).astype(np.float32)
    t = rng.normal(0.0, 1.0, n).astype(np.float32)
    return net, p.astype(np.float64), x, t


@pytest.mark.parametrize("n_in,hidden,layers,n", CASES)
def test_forward_against_oracle(torch_cuda, n_in, hidden, layers, n):
    torch = torch_cuda
    _print(f"case forward n_in={n_in} hidden={hidden} layers={layers} n={n}")
    net, p, x, _ = _setup(torch, n_in, hidden, layers, n, seed=11 + n)
    y = net.forward(torch.from_numpy(x).cuda()).cpu().numpy().astype(np.float64)
    yb, _, _ = M.forward(p, x, n_in, hidden, layers, bf16_acts=True)
    y64, _, _ = M.forward(p, x, n_in, hidden, layers)
    eb, e64 = _rel(y, yb), _rel(y, y64)
    _print(f"  rel vs bf16-operand oracle {eb:.2e}, vs fp64 oracle {e64:.2e}")
    assert eb <= 2e-3 and e64 <= 3e-2


@pytest.mark.parametrize("n_in,hidden,layers,n", CASES)
def test_gradients_against_oracle(torch_cuda, n_in, hidden, layers, n):
    torch = torch_cuda
    _print(f"case gradients n_in={n_in} hidden={hidden} layers={layers} n={n}")
    net, p, x, t = _setup(torch, n_in, hidden, layers, n, seed=29 + n)
    loss, g = net.gradients(torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda())
    lb, gb = M.loss_and_grad(p, x, t, n_in, hidden, layers, bf16_acts=True)
    l64, g64 = M.loss_and_grad(p, x, t, n_in, hidden, layers)
    assert abs(loss - lb) <= 2e-3 * lb
    k = 0
    for l, (o, i) in enumerate(M.layer_shapes(n_in, hidden, layers)):
        for name, size in (("W", o * i), ("b", o)):
            sl = slice(k, k + size)
            eb, e64 = _rel(g[sl], gb[sl]), _rel(g[sl], g64[sl])
            _print(f"  layer {l} {name}: rel vs bf16-operand oracle {eb:.2e}, vs fp64 {e64:.2e}")
            assert eb <= 1.5e-2 and e64 <= 6e-2, (l, name)
            k += size
    assert k == g.size


def test_first_adam_step_moves_by_lr_sign(torch_cuda):
    # after one Adam step from zero moments, m_hat = g and v_hat = g^2: p1 = p0 - lr g / (|g| + eps)
    torch = torch_cuda
    net, p0, x, t = _setup(torch, 4, 64, 2, 300, seed=3)
    xd, td = torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda()
    _, g = net.gradients(xd, td)
    lr = 1e-3
    net.train_step(xd, td, lr)
    p1 = net.params().astype(np.float64)
    g = g.astype(np.float64)
    expect = p0 - lr * g / (np.abs(g) + 1e-8)
    assert np.abs(p1 - expect).max() <= 1e-6


def test_training_reduces_loss(torch_cuda):
    torch = torch_cuda
    from paper_1902_10432_amd.surrogate import Surrogate
    rng = np.random.default_rng(7)
    n = 4096
    x = rng.uniform(-1.0, 1.0, (n, 4)).astype(np.float32)
    t = (np.sin(2 * x[:, 0]) * np.cos(x[:, 1]) + 0.5 * x[:, 2] * x[:, 3]).astype(np.float32)
    xd, td = torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda()
    net = Surrogate(4, 128, 4, max_batch=n, seed=1)
    first = net.train_step(xd, td, 2e-3, want_loss=True)
    for _ in range(400):
        net.train_step(xd, td, 2e-3)
    last = net.train_step(xd, td, 2e-3, want_loss=True)
    _print(f"  loss {first:.4e} -> {last:.4e}")
    assert last < 0.02 * first
    y = net.forward(xd).cpu().numpy()
    assert _rel(y, t) < 0.15


@pytest.mark.parametrize("n", [1, 63, 1000, 4097])
def test_fused_inference_matches_layered_forward(torch_cuda, n):
    """Inference at width 128 runs the whole network in one kernel; the loss the gradient call
    reports (its layer-by-layer forward) against the fused outputs as targets is the mean squared
    difference of the two forward passes: identical products, output sums in another order."""
    torch = torch_cuda
    net, _, x, _ = _setup(torch, 4, 128, 4, n, seed=41 + n)
    xd = torch.from_numpy(x).cuda()
    y = net.forward(xd)
    loss, _ = net.gradients(xd, y)
    rms = float(torch.sqrt((y ** 2).mean()))
    _print(f"  n={n}: rms diff {loss ** 0.5:.2e} of rms {rms:.2e}")
    assert loss ** 0.5 <= 1e-5 * rms
