"""The manufactured-solution case (paper Sec. "Method of manufactured solutions") on the
oracle: the closed-form error of the discrete steady state, which the GPU study is
checked against, is pinned here by marching the oracle's own stencils and RK3 to
T = 100, including grids narrower than the stencil (indices wrap more than once)."""
import math

import numpy as np
import pytest

import oracle
from test_gpu_scalar import mms_discrete_steady_error

U0, U1, K = 1.0, -0.5, 0.75


def oracle_mms_error(order, n, T=100.0):
    h = 2 * np.pi / n
    x = np.arange(n) * h
    X1, X0 = np.meshgrid(x, x, indexing="ij")
    S = -(U0 * np.cos(X0) * np.cos(X1) - U1 * np.sin(X0) * np.sin(X1) + 2 * K * np.sin(X0) * np.cos(X1))
    p = oracle.Params(n=(n, n, 1), order=order, length=(2 * np.pi, 2 * np.pi, 1.0))

    def rhs(y):
        f = y.reshape(1, n, n)
        out = K * (oracle.d2(f, 0, p) + oracle.d2(f, 1, p)) - U0 * oracle.d1(f, 0, p) - U1 * oracle.d1(f, 1, p)
        return (out[0] - S).ravel()

    dt = 0.025 / (abs(U0) / h + abs(U1) / h)
    phi = oracle.rk3_generic(np.zeros(n * n), dt, int(math.ceil(T / dt)), rhs)
    e = phi.reshape(n, n) - np.sin(X0) * np.cos(X1)
    return math.sqrt(np.mean(e * e))


@pytest.mark.parametrize("order,n", [(2, 8), (4, 8), (12, 4), (8, 16)])
def test_discrete_steady_error_closed_form(oracle_mod, order, n):
    """Agreement to rounding: the closed form loses ~1e-16 absolute in A - 1."""
    got = oracle_mms_error(order, n)
    ref = mms_discrete_steady_error(order, n)
    assert abs(got - ref) <= 1e-9 * ref + 1e-14, (got, ref)


@pytest.mark.parametrize("order", [8, 12])
def test_wide_stencil_modified_wavenumber_on_four_points(oracle_mod, order):
    """D sin x = s cos x and D2 sin x = -t sin x on 4 points, with the stencil wrapping
    the grid more than once (s, t: the modified wavenumbers of the weights at h = pi/2)."""
    from oracle import stencil
    n, h = 4, np.pi / 2
    x = np.arange(n) * h
    f = np.sin(x)[None, None, :]
    p = oracle.Params(n=(n, 1, 1), order=order, length=(2 * np.pi, 1.0, 1.0))
    a = [float(v) for v in stencil.first_derivative_weights(order)]
    c0, c = stencil.second_derivative_weights(order)
    s = sum(2 * a[m - 1] * math.sin(m * h) for m in range(1, len(a) + 1)) / h
    t = -(float(c0) + sum(2 * float(c[m - 1]) * math.cos(m * h) for m in range(1, len(c) + 1))) / h ** 2
    assert np.allclose(oracle.d1(f, 0, p)[0, 0], s * np.cos(x), atol=1e-14)
    assert np.allclose(oracle.d2(f, 0, p)[0, 0], -t * np.sin(x), atol=1e-13)
