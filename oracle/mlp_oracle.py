"""Plain FP64 NumPy reference of the bridge-force surrogate network (test infrastructure).

TEST INFRASTRUCTURE ONLY: used by the test suite to check the GPU network's forward pass and
parameter gradients; the product path never imports it.

The network is the multilayer perceptron n_in -> hidden x layers -> 1 with SiLU activations,
z = a W^T + b per layer, parameters packed per layer as W [out][in] then b [out], trained on the
mean-squared error (1/n) sum (y - t)^2.  The backward pass is the chain rule written out; its pin
is a central finite-difference check of the loss (tests/test_oracle_mlp.py).
"""
from __future__ import annotations

import numpy as np


def layer_shapes(n_in: int, hidden: int, layers: int):
    shapes = []
    for l in range(layers + 1):
        i = n_in if l == 0 else hidden
        o = 1 if l == layers else hidden
        shapes.append((o, i))
    return shapes


def unpack(params: np.ndarray, n_in: int, hidden: int, layers: int):
    out, k = [], 0
    for o, i in layer_shapes(n_in, hidden, layers):
        W = params[k:k + o * i].reshape(o, i)
        k += o * i
        b = params[k:k + o]
        k += o
        out.append((W, b))
    assert k == params.size
    return out


def silu(z):
    return z / (1.0 + np.exp(-z))


def silu_grad(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def forward(params, x, n_in, hidden, layers, bf16_acts=False):
    """Output [n] and the pre-activations / activations of every layer.

    bf16_acts: round the input and every hidden activation to BF16 (through FP32) before it
    enters the next product, as a network whose matrix operands are stored in BF16 does; the
    products and sums themselves stay exact in FP64."""
    Ws = unpack(np.asarray(params, dtype=np.float64), n_in, hidden, layers)
    rnd = to_bf16 if bf16_acts else (lambda v: v)
    a = rnd(np.asarray(x, dtype=np.float64))
    zs, acts = [], [a]
    for l, (W, b) in enumerate(Ws):
        z = a @ W.T + b
        zs.append(z)
        a = z if l == len(Ws) - 1 else rnd(silu(z))
        acts.append(a)
    return a[:, 0], zs, acts


def loss_and_grad(params, x, t, n_in, hidden, layers, bf16_acts=False):
    """Mean-squared-error loss and its gradient with respect to the packed parameters.

    With bf16_acts the forward pass rounds its operands as in forward(), and the backward pass
    takes each rounding as the identity (the gradient a BF16-operand network computes)."""
    params = np.asarray(params, dtype=np.float64)
    Ws = unpack(params, n_in, hidden, layers)
    y, zs, acts = forward(params, x, n_in, hidden, layers, bf16_acts)
    t = np.asarray(t, dtype=np.float64)
    n = y.size
    e = y - t
    loss = float(np.mean(e * e))
    dz = (2.0 * e / n)[:, None]
    grads = [None] * len(Ws)
    for l in range(len(Ws) - 1, -1, -1):
        W, _ = Ws[l]
        grads[l] = (dz.T @ acts[l], dz.sum(axis=0))
        if l == 0:
            break
        da = dz @ W
        dz = da * silu_grad(zs[l - 1])
    flat = np.concatenate([np.concatenate([gW.ravel(), gb]) for gW, gb in grads])
    return loss, flat


def to_bf16(a: np.ndarray) -> np.ndarray:
    """Round FP32 values to the nearest BF16 (ties to even), returned as float64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)
