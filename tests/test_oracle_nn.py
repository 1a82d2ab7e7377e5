"""Pins of the learned-closure oracle (oracle/nn.py)."""
import math

import numpy as np
import pytest

from oracle import nn


def test_conv3d_matches_scipy_wrap_correlation():
    from scipy.ndimage import correlate
    rng = np.random.default_rng(0)
    x = rng.standard_normal((2, 3, 5, 6, 7))
    W = rng.standard_normal((4, 3, 3, 3, 3))
    b = rng.standard_normal(4)
    out = nn.conv3d(x, W, b)
    for bb in range(2):
        for o in range(4):
            ref = b[o] + sum(correlate(x[bb, i], W[o, i], mode="wrap") for i in range(3))
            assert np.abs(out[bb, o] - ref).max() < 1e-12


def test_conv3d_delta_kernel_is_a_shift():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((1, 1, 6, 6, 6))
    W = np.zeros((1, 1, 3, 3, 3))
    W[0, 0, 2, 0, 1] = 1.0       # dz = +1, dy = -1, dx = 0
    out = nn.conv3d(x, W, np.zeros(1))
    assert np.array_equal(out, np.roll(x, shift=(-1, 1, 0), axis=(2, 3, 4)))


def _fd_check(f, p, grad, eps=1e-6, samples=12, seed=0):
    rng = np.random.default_rng(seed)
    flat = p.reshape(-1)
    g = grad.reshape(-1)
    for idx in rng.choice(flat.size, size=min(samples, flat.size), replace=False):
        old = flat[idx]
        flat[idx] = old + eps
        fp = f()
        flat[idx] = old - eps
        fm = f()
        flat[idx] = old
        num = (fp - fm) / (2 * eps)
        assert abs(num - g[idx]) <= 1e-7 * max(1.0, abs(num)) + 1e-9, (idx, num, g[idx])


def test_network_gradients_match_finite_differences():
    rng = np.random.default_rng(2)
    params = nn.init_params(rng, channels=(2, 3, 3, 2))
    for W, b in params:
        b[:] = rng.standard_normal(b.shape) * 0.1
    x = rng.standard_normal((2, 2, 4, 5, 4))
    t = rng.standard_normal((2, 2, 4, 5, 4))

    def loss():
        y, _ = nn.forward(params, x)
        return nn.mse(y, t)[0]

    y, cache = nn.forward(params, x)
    _, dy = nn.mse(y, t)
    grads = nn.backward(params, cache, dy)
    for (W, b), (dW, db) in zip(params, grads):
        _fd_check(loss, W, dW)
        _fd_check(loss, b, db)


def test_bwd_data_matches_finite_differences():
    rng = np.random.default_rng(3)
    x = rng.standard_normal((1, 2, 4, 4, 5))
    W = rng.standard_normal((3, 2, 3, 3, 3))
    b = rng.standard_normal(3)
    r = rng.standard_normal((1, 3, 4, 4, 5))

    def loss():
        return float(np.sum(nn.conv3d(x, W, b) * r))

    _fd_check(loss, x, nn.conv3d_bwd_data(r, W), samples=20)


def test_gelu_values_and_derivative():
    xs = np.array([-3.0, -1.0, -0.2, 0.0, 0.5, 2.0])
    ref = np.array([0.5 * v * (1 + math.erf(v / math.sqrt(2))) for v in xs])
    assert np.abs(nn.gelu(xs) - ref).max() < 1e-15
    h = 1e-6
    num = (nn.gelu(xs + h) - nn.gelu(xs - h)) / (2 * h)
    assert np.abs(nn.gelu_grad(xs) - num).max() < 1e-8


def test_adam_first_step_closed_form():
    # from zero moments, the bias-corrected first step is lr * g / (|g| + eps)
    rng = np.random.default_rng(4)
    p = rng.standard_normal(10)
    g = rng.standard_normal(10)
    lr = 1e-3
    p1, m, v = nn.adam_step(p.copy(), g, np.zeros(10), np.zeros(10), 1, lr)
    assert np.abs(p1 - (p - lr * g / (np.abs(g) + 1e-8))).max() < 1e-15


@pytest.mark.parametrize("k", [1, 3, 5])
def test_box_filter_transfer_function(k):
    n, ratio = 32, 4
    x = 2 * np.pi * np.arange(n) / n
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    f = np.cos(k * X + 0.3) * np.ones_like(Y)
    h = 2 * np.pi / n
    G = 0.25 + 0.5 * np.cos(k * h) + 0.25 * np.cos(2 * k * h)
    out = nn.box_filter(f[None], ratio)[0]
    ref = G * np.cos(k * X[::ratio, ::ratio, ::ratio] + 0.3)
    assert np.abs(out - ref).max() < 1e-13


def test_box_filter_conserves_mean():
    rng = np.random.default_rng(5)
    f = rng.standard_normal((5, 16, 16, 16))
    out = nn.box_filter(f, 4)
    assert np.abs(out.mean(axis=(1, 2, 3)) - f.mean(axis=(1, 2, 3))).max() < 1e-14
