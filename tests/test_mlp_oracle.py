"""Pins of the predictor network's float64 reference (oracle/mlp_oracle.py):
its gradient against central finite differences of its loss, its forward
pass against hand-derivable cases, and its bfloat16 rounding against the
bit patterns of the format."""
import numpy as np
import pytest

from oracle import mlp_oracle as m


def _random(seed, n=40):
    rng = np.random.default_rng(seed)
    theta = rng.normal(0.0, 0.3, m.NPARAM)
    X = np.log1p(rng.integers(0, 50, (n, 64)).astype(np.float64))
    y = rng.normal(0.0, 1.0, n)
    return theta, X, y


@pytest.mark.parametrize("seed,tau", [(0, 0.9), (1, 0.5), (2, 0.75)])
def test_grad_matches_finite_differences(seed, tau):
    theta, X, y = _random(seed)
    g = m.grad(theta, X, y, tau)
    rng = np.random.default_rng(100 + seed)
    idx = np.concatenate([rng.integers(0, m.NPARAM, 40), [4096, 4159, 8256, 8320, 8383, 8384]])
    eps = 1e-6
    for i in idx:
        t1, t2 = theta.copy(), theta.copy()
        t1[i] += eps
        t2[i] -= eps
        fd = (m.loss(t1, X, y, tau) - m.loss(t2, X, y, tau)) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-6 + 1e-5 * abs(fd), (i, fd, g[i])


def test_forward_identity_network():
    # W1 = W2 = I, zero biases, w3 = 1: yhat = sum of the (non-negative) features
    theta = m.pack({"W1": np.eye(64), "b1": np.zeros(64), "W2": np.eye(64), "b2": np.zeros(64),
                    "w3": np.ones(64), "b3": np.array([0.5])})
    X = np.arange(128, dtype=np.float64).reshape(2, 64) / 10.0
    yhat = m.forward(theta, X)[4]
    assert np.allclose(yhat, X.sum(axis=1) + 0.5)
    # ReLU: negative inputs contribute nothing
    assert np.allclose(m.forward(theta, -X)[4], 0.5)


def test_pinball_loss_values():
    theta = m.pack({"W1": np.zeros((64, 64)), "b1": np.zeros(64), "W2": np.zeros((64, 64)), "b2": np.zeros(64),
                    "w3": np.zeros(64), "b3": np.array([1.0])})
    X = np.zeros((2, 64))
    # yhat = 1 for both rows; y = 3 (under-predicted by 2), y = 0 (over by 1)
    assert np.isclose(m.loss(theta, X, np.array([3.0, 0.0]), 0.9), (0.9 * 2 + 0.1 * 1) / 2)
    g = m.grad(theta, X, np.array([3.0, 0.0]), 0.9)
    assert np.isclose(g[-1], (-0.9 + 0.1) / 2)


def test_bf16_round():
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, 1.0 + 2 ** -7, -2.5, 0.0, 3.0e38])
    want = np.array([1.0, 1.0, 1.0 + 2 ** -7, 1.0 + 2 ** -7, -2.5, 0.0, np.float32(3.0e38).view(np.uint32)])
    got = m.bf16_round(vals)
    assert got[0] == 1.0 and got[1] == 1.0          # tie rounds to even
    assert got[2] == 1.0 + 2 ** -7 and got[3] == 1.0 + 2 ** -7
    assert got[4] == -2.5 and got[5] == 0.0
    assert (np.float32(got[6]).view(np.uint32) & 0xFFFF) == 0
    assert want.shape == got.shape
