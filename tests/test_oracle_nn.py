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


def test_conv3d_at_points_equals_whole_grid():
    """The point-by-point gather form equals the rolled whole-grid form everywhere,
    including the wrapped faces and batch entries beyond the first."""
    rng = np.random.default_rng(6)
    x = rng.standard_normal((3, 4, 5, 6, 7))
    W = rng.standard_normal((2, 4, 3, 3, 3))
    b = rng.standard_normal(2)
    full = nn.conv3d(x, W, b)
    pts = [(bb, z, y, xx) for bb in range(3) for z in range(5) for y in range(6) for xx in range(7)]
    got = nn.conv3d_at_points(x, W, b, pts)
    ref = np.array([full[bb, :, z, y, xx] for bb, z, y, xx in pts])
    assert np.abs(got - ref).max() < 1e-12


def test_conv3d_bwd_data_at_points_equals_whole_grid():
    rng = np.random.default_rng(7)
    dy = rng.standard_normal((2, 3, 4, 5, 6))
    W = rng.standard_normal((3, 2, 3, 3, 3))
    full = nn.conv3d_bwd_data(dy, W)
    pts = [(bb, z, y, xx) for bb in range(2) for z in range(4) for y in range(5) for xx in range(6)]
    got = nn.conv3d_bwd_data_at_points(dy, W, pts)
    ref = np.array([full[bb, :, z, y, xx] for bb, z, y, xx in pts])
    assert np.abs(got - ref).max() < 1e-12


def test_adam_constant_gradient_closed_form():
    """With a constant gradient g the bias-corrected moments are exactly g and g^2 at
    every step (m_t = (1 - b1^t) g, v_t = (1 - b2^t) g^2), so each of the first three
    steps moves p by lr g / (|g| + eps).  A bias correction with the wrong exponent
    (for example always that of step 1) fails at t = 2."""
    rng = np.random.default_rng(8)
    p0 = rng.standard_normal(16)
    g = rng.standard_normal(16)
    lr = 1e-3
    p, m, v = p0.copy(), np.zeros(16), np.zeros(16)
    for t in (1, 2, 3):
        p, m, v = nn.adam_step(p, g, m, v, t, lr)
        assert np.abs(p - (p0 - t * lr * g / (np.abs(g) + 1e-8))).max() < 1e-14, t


def test_adam_second_step_closed_forms():
    """Second step after g1, by hand from the definitions:
    g2 = 0:    m2^ = b1/(1+b1) g1, v2^ = b2/(1+b2) g1^2;
    g2 = -g1:  m2^ = -(1-b1)/(1+b1) g1, v2^ = g1^2."""
    rng = np.random.default_rng(9)
    g1 = rng.standard_normal(12)
    lr, b1, b2, eps = 2e-3, 0.9, 0.999, 1e-8
    p0 = rng.standard_normal(12)
    p1, m1, v1 = nn.adam_step(p0.copy(), g1, np.zeros(12), np.zeros(12), 1, lr)
    p2, _, _ = nn.adam_step(p1.copy(), np.zeros(12), m1.copy(), v1.copy(), 2, lr)
    ref = p1 - lr * (b1 / (1 + b1)) * g1 / (np.sqrt(b2 / (1 + b2)) * np.abs(g1) + eps)
    assert np.abs(p2 - ref).max() < 1e-14
    p2, m2, v2 = nn.adam_step(p1.copy(), -g1, m1.copy(), v1.copy(), 2, lr)
    ref = p1 + lr * ((1 - b1) / (1 + b1)) * g1 / (np.abs(g1) + eps)
    assert np.abs(p2 - ref).max() < 1e-14
    # third step with g3 = g1 after (g1, -g1): m3 = (1-b1)(b1^2 - b1 + 1) g1
    p3, _, _ = nn.adam_step(p2.copy(), g1, m2.copy(), v2.copy(), 3, lr)
    mh = (1 - b1) * (b1 * b1 - b1 + 1) / (1 - b1 ** 3) * g1
    vh = (1 - b2) * (b2 * b2 + b2 + 1) / (1 - b2 ** 3) * g1 * g1
    assert np.abs(p3 - (p2 - lr * mh / (np.sqrt(vh) + eps))).max() < 1e-14


def test_remove_box_mean_on_constant_and_zero_mean_fields():
    # a constant field (its own value per sample and field) has nothing left; a field
    # of whole periods of sines has zero box mean and is unchanged; the two add
    n = 12
    rng = np.random.default_rng(3)
    const = rng.uniform(-5, 5, size=(2, 5, 1, 1, 1)) * np.ones((2, 5, n, n, n))
    x = np.arange(n) * 2 * np.pi / n
    wave = np.sin(x)[None, None, None, None, :] * np.cos(2 * x)[None, None, :, None, None] * np.ones((2, 5, n, n, n))
    wave *= rng.uniform(0.5, 2.0, size=(2, 5, 1, 1, 1))
    assert np.abs(nn.remove_box_mean(const)).max() <= 1e-14
    assert np.abs(nn.remove_box_mean(wave) - wave).max() <= 1e-14
    assert np.abs(nn.remove_box_mean(const + wave) - wave).max() <= 1e-13
