"""Plain numpy (float64) reference of the search-radius predictor's network.

TEST INFRASTRUCTURE ONLY: the GPU tests call it to check the HIP forward and
gradient kernels; the product path never does.  It shares no code with the
HIP library.

The predictor is not part of the paper: it bounds the k-NN search of Sec. 5
(which the paper does over a fixed block of 26 neighbouring voxels) by a
radius predicted from the occupancy around a cell.  The network is a
multilayer perceptron 64 -> 64 -> 64 -> 1 with ReLU after the two hidden
layers; parameters are stored flat, in this order:

    W1 [64 in][64 out], b1 [64], W2 [64][64], b2 [64], w3 [64], b3 [1]

The loss is the mean pinball (quantile) loss at level tau of the prediction
yhat against the target y, tau * max(y - yhat, 0) + (1 - tau) * max(yhat - y, 0),
which pushes predictions above the targets for tau > 1/2.
"""
from __future__ import annotations

import numpy as np

NPARAM = 64 * 64 + 64 + 64 * 64 + 64 + 64 + 1
_SHAPES = [("W1", (64, 64)), ("b1", (64,)), ("W2", (64, 64)), ("b2", (64,)), ("w3", (64,)), ("b3", (1,))]


def unpack(theta):
    theta = np.asarray(theta, dtype=np.float64)
    assert theta.shape == (NPARAM,)
    out, o = {}, 0
    for name, shape in _SHAPES:
        size = int(np.prod(shape))
        out[name] = theta[o:o + size].reshape(shape)
        o += size
    return out


def pack(parts):
    return np.concatenate([np.asarray(parts[name], dtype=np.float64).ravel() for name, _ in _SHAPES])


def bf16_round(x):
    """Round float64 values to bfloat16 (round to nearest, ties to even),
    returned as float64: the precision of the GPU's matrix operands."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _id(x):
    return x


def forward(theta, X, bf16_operands=False):
    """Hidden activations and outputs: X [n, 64] -> (Z1, H1, Z2, H2, yhat).

    With bf16_operands the operands of the two matrix products (X, W1, H1,
    W2) are rounded to bfloat16 first, as the GPU's matrix cores take them;
    everything else stays float64."""
    p = unpack(theta)
    r = bf16_round if bf16_operands else _id
    X = np.asarray(X, dtype=np.float64)
    Z1 = r(X) @ r(p["W1"]) + p["b1"]
    H1 = np.maximum(Z1, 0.0)
    Z2 = r(H1) @ r(p["W2"]) + p["b2"]
    H2 = np.maximum(Z2, 0.0)
    yhat = H2 @ p["w3"] + p["b3"][0]
    return Z1, H1, Z2, H2, yhat


def loss(theta, X, y, tau):
    yhat = forward(theta, X)[4]
    r = np.asarray(y, dtype=np.float64) - yhat
    return float(np.mean(np.where(r > 0, tau * r, (tau - 1.0) * r)))


def grad(theta, X, y, tau, bf16_operands=False):
    """Gradient of loss() by the chain rule, layer by layer from the output.

    With bf16_operands the operands of every matrix product, forward and
    backward (X, W1, H1, W2, dZ2, dZ1), are rounded to bfloat16 first."""
    p = unpack(theta)
    r = bf16_round if bf16_operands else _id
    X = np.asarray(X, dtype=np.float64)
    n = X.shape[0]
    Z1, H1, Z2, H2, yhat = forward(theta, X, bf16_operands)
    res = np.asarray(y, dtype=np.float64) - yhat
    dy = np.where(res > 0, -tau, np.where(res < 0, 1.0 - tau, 0.0)) / n
    g = {"w3": H2.T @ dy, "b3": np.array([dy.sum()])}
    dZ2 = np.outer(dy, p["w3"]) * (Z2 > 0)
    g["W2"] = r(H1).T @ r(dZ2)
    g["b2"] = dZ2.sum(axis=0)
    dZ1 = (r(dZ2) @ r(p["W2"]).T) * (Z1 > 0)
    g["W1"] = r(X).T @ r(dZ1)
    g["b1"] = dZ1.sum(axis=0)
    return pack(g)
