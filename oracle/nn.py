"""FP64 reference of the learned-closure pieces: box filter, periodic 3D convolution
network (conv -> GELU -> conv -> GELU -> conv), mean-squared error, Adam.

TEST INFRASTRUCTURE ONLY (part of the oracle): only tests, the smoke check and the
CPU-baseline leg of the benchmark may use it.  Written from the definitions with numpy:
no blocking, fusion or reordering, layouts planar [batch][channel][z][y][x].

Pins (tests/test_oracle_nn.py): the convolution against scipy.ndimage.correlate with
periodic wrap, every hand-derived gradient against central finite differences in
FP64, Adam's first step against its closed form, the filter's transfer function
on Fourier modes, and the box-mean removal on constant and zero-mean fields.
"""
import math

import numpy as np

SQRT2 = math.sqrt(2.0)
INV_SQRT_2PI = 1.0 / math.sqrt(2.0 * math.pi)


def _erf(x):
    from scipy.special import erf
    return erf(x)


# ----------------------------------------------------------------------------- filter
def box_filter(f, ratio=4):
    """Separable centred trapezoidal box filter of width ratio*h on a periodic grid,
    sampled at every `ratio`-th point (coarse point i sits on fine point ratio*i).

    Weights along each axis: 1/(2 ratio) at offsets +-ratio/2, 1/ratio in between.
    f: array whose last three axes are (z, y, x) with sizes divisible by ratio.
    """
    if ratio % 2:
        raise ValueError("ratio must be even")
    h = ratio // 2
    w = {o: 1.0 / ratio for o in range(-h + 1, h)}
    w[-h] = w[h] = 1.0 / (2 * ratio)
    g = np.asarray(f, dtype=np.float64)
    for ax in (-1, -2, -3):
        acc = np.zeros_like(g)
        for o, wo in sorted(w.items()):
            acc += wo * np.roll(g, -o, axis=ax)
        g = acc
    return g[..., ::ratio, ::ratio, ::ratio].copy()


# ----------------------------------------------------------------------------- network
def conv3d(x, W, b):
    """Periodic 3x3x3 cross-correlation: x [B][Ci][n][n][n], W [Co][Ci][3][3][3], b [Co].
    out[b,o,z,y,x] = b[o] + sum_{i,dz,dy,dx} W[o,i,dz+1,dy+1,dx+1] x[b,i,z+dz,y+dy,x+dx]."""
    B, Ci = x.shape[:2]
    Co = W.shape[0]
    out = np.zeros((B, Co) + x.shape[2:])
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                xs = np.roll(x, shift=(-dz, -dy, -dx), axis=(2, 3, 4))
                out += np.einsum("oi,bizyx->bozyx", W[:, :, dz + 1, dy + 1, dx + 1], xs)
    return out + b[None, :, None, None, None]


def conv3d_bwd_data(dy, W):
    """d(loss)/dx for the convolution above, given d(loss)/d(out) = dy."""
    dx_ = np.zeros((dy.shape[0], W.shape[1]) + dy.shape[2:])
    for dz in (-1, 0, 1):
        for dyo in (-1, 0, 1):
            for dxo in (-1, 0, 1):
                contrib = np.einsum("oi,bozyx->bizyx", W[:, :, dz + 1, dyo + 1, dxo + 1], dy)
                dx_ += np.roll(contrib, shift=(dz, dyo, dxo), axis=(2, 3, 4))
    return dx_


def conv3d_bwd_weight(x, dy):
    """(dW, db) for the convolution above."""
    Co, Ci = dy.shape[1], x.shape[1]
    dW = np.zeros((Co, Ci, 3, 3, 3))
    for dz in (-1, 0, 1):
        for dyo in (-1, 0, 1):
            for dxo in (-1, 0, 1):
                xs = np.roll(x, shift=(-dz, -dyo, -dxo), axis=(2, 3, 4))
                # the sum over samples and points as one library contraction
                dW[:, :, dz + 1, dyo + 1, dxo + 1] = np.tensordot(dy, xs, axes=([0, 2, 3, 4], [0, 2, 3, 4]))
    db = dy.sum(axis=(0, 2, 3, 4))
    return dW, db


def _taps():
    return [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def conv3d_at_points(x, W, b, pts):
    """The convolution above evaluated only at sample/point pairs pts = [(b, z, y, x)]:
    returns out[k, o] = b[o] + sum_{i,dz,dy,dx} W[o,i,dz+1,dy+1,dx+1] x[b_k,i,z_k+dz,y_k+dy,x_k+dx]
    (indices wrap), gathered point by point."""
    pts = np.asarray(pts, dtype=np.int64)
    n = x.shape[2:]
    out = np.tile(np.asarray(b, dtype=np.float64), (len(pts), 1))
    for dz, dy, dx in _taps():
        nb = x[pts[:, 0], :, (pts[:, 1] + dz) % n[0], (pts[:, 2] + dy) % n[1], (pts[:, 3] + dx) % n[2]]
        out += nb @ W[:, :, dz + 1, dy + 1, dx + 1].T
    return out


def conv3d_bwd_data_at_points(dy, W, pts):
    """conv3d_bwd_data(dy, W) at pts = [(b, z, y, x)]: out[k, i] = sum_{o,dz,dy,dx}
    W[o,i,dz+1,dy+1,dx+1] dy[b_k, o, z_k-dz, y_k-dy, x_k-dx] (the point the tap reaches
    this one from), gathered point by point."""
    pts = np.asarray(pts, dtype=np.int64)
    n = dy.shape[2:]
    out = np.zeros((len(pts), W.shape[1]))
    for dz, dyo, dx in _taps():
        nb = dy[pts[:, 0], :, (pts[:, 1] - dz) % n[0], (pts[:, 2] - dyo) % n[1], (pts[:, 3] - dx) % n[2]]
        out += nb @ W[:, :, dz + 1, dyo + 1, dx + 1]
    return out


def gelu(x):
    """Exact GELU: x * Phi(x) with the Gaussian CDF written with erf."""
    return 0.5 * x * (1.0 + _erf(x / SQRT2))


def gelu_grad(x):
    """d GELU / dx = Phi(x) + x phi(x)."""
    return 0.5 * (1.0 + _erf(x / SQRT2)) + x * INV_SQRT_2PI * np.exp(-0.5 * x * x)


def init_params(rng, channels=(5, 32, 32, 5)):
    """He-style uniform initialisation from a numpy Generator (the draws are the input)."""
    params = []
    for ci, co in zip(channels[:-1], channels[1:]):
        bound = math.sqrt(6.0 / (ci * 27))
        params.append((rng.uniform(-bound, bound, (co, ci, 3, 3, 3)), np.zeros(co)))
    return params


def forward(params, x):
    """Network output and the cache needed for the backward pass."""
    cache = []
    h = x
    for li, (W, b) in enumerate(params):
        pre = conv3d(h, W, b)
        cache.append((h, pre))
        h = gelu(pre) if li < len(params) - 1 else pre
    return h, cache


def remove_box_mean(y):
    """Conservative form of a closure term: each field of each sample, planar
    [batch][field][z][y][x], minus its mean over the box.  The exact closure term
    F R_f - R_c(F q_f) has zero box mean, because both residuals are in conservative
    form (paper Sec. "3D Taylor-Green vortex") and the filter keeps totals."""
    y = np.asarray(y, dtype=np.float64)
    return y - y.mean(axis=(2, 3, 4), keepdims=True)


def mse(y, t):
    """Mean squared error over every element, and its gradient."""
    d = y - t
    return float(np.mean(d * d)), 2.0 * d / d.size


def backward(params, cache, dy):
    """Gradients [(dW, db)] of the loss for every layer given d(loss)/d(output)."""
    grads = [None] * len(params)
    g = dy
    for li in range(len(params) - 1, -1, -1):
        W, _ = params[li]
        h_in, pre = cache[li]
        if li < len(params) - 1:
            g = g * gelu_grad(pre)
        grads[li] = conv3d_bwd_weight(h_in, g)
        if li > 0:
            g = conv3d_bwd_data(g, W)
    return grads


def adam_step(p, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba), bias-corrected; returns new (p, m, v)."""
    m = beta1 * m + (1 - beta1) * g
    v = beta2 * v + (1 - beta2) * g * g
    mh = m / (1 - beta1 ** t)
    vh = v / (1 - beta2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
