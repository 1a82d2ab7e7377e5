"""Pins of the oracle's low-storage RK3 (paper Sec. "Discretisation schemes") and of the
1D wave test case (paper Sec. "Propagation of a wave")."""
import json
import math
import os

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_linear_stability_polynomial(oracle_mod):
    # On y' = L y every 3-stage third-order RK gives y1 = (1 + z + z^2/2 + z^3/6) y0.
    # A 2x2 rotation-plus-decay block makes z complex.
    lam = complex(-0.7, 2.3)
    Lm = np.array([[lam.real, -lam.imag], [lam.imag, lam.real]])
    dt = 0.37
    y0 = np.array([0.6, -1.1])
    y1 = oracle.rk3_generic(y0, dt, 1, lambda y: Lm @ y)
    z = lam * dt
    R = 1 + z + z * z / 2 + z ** 3 / 6
    w = R * complex(y0[0], y0[1])
    assert abs(y1[0] - w.real) < 1e-14 and abs(y1[1] - w.imag) < 1e-14


def test_third_order_on_nonlinear_ode(oracle_mod):
    # y' = y^2, y(0) = 1/2  ->  y(t) = 1/(2 - t).  Halving dt divides the global error by 8
    # only if every third-order condition (including b.c^2 = 1/3) holds.
    T = 1.0
    errs = []
    for nsteps in (20, 40, 80, 160):
        y = oracle.rk3_generic(np.array([0.5]), T / nsteps, nsteps, lambda y: y * y)
        errs.append(abs(y[0] - 1.0 / (2.0 - T)))
    ratios = [errs[i] / errs[i + 1] for i in range(3)]
    assert all(abs(r - 8.0) < 0.6 for r in ratios), ratios


def test_first_order_would_fail():
    # Guard on the test above: a forward-Euler step gives ratio 2, not 8.
    errs = []
    for nsteps in (20, 40):
        y, dt = 0.5, 1.0 / nsteps
        for _ in range(nsteps):
            y = y + dt * y * y
        errs.append(abs(y - 1.0))
    assert abs(errs[0] / errs[1] - 2.0) < 0.3


def test_wave1d_paper_case(oracle_mod):
    """1D wave: 8th order, RK3, c = 0.5, dx = 1e-3, dt = 4e-4, to t = 1.

    The oracle's discrete solution equals Im[R(z)^n e^{ikx}] with z = -i c dt k*
    (k* the modified wavenumber), and its error against sin(2 pi (x - c t)) is
    of the order the paper prints (1e-10)."""
    g = json.load(open(os.path.join(GOLDEN, "wave1d.json")))
    c, dx, dt, T, order = g["c"], g["dx"], g["dt"], g["t_end"], g["order"]
    n = int(round(1.0 / dx))
    nsteps = int(round(T / dt))
    p = oracle.Params(n=(n, 1, 1), order=order, length=(1.0, 1.0, 1.0))
    # a 1-point y/z extent: only x-derivatives are taken
    x = np.arange(n) * dx
    phi0 = np.sin(2 * np.pi * x)

    def f(y):
        return -c * oracle.d1(y.reshape(1, 1, n), 0, p).ravel()

    phi = oracle.rk3_generic(phi0, dt, nsteps, f)
    k = 2 * np.pi
    r = order // 2
    from oracle.stencil import first_derivative_weights
    a = [float(v) for v in first_derivative_weights(order)]
    ks = 2 / dx * sum(a[m - 1] * math.sin(m * k * dx) for m in range(1, r + 1))
    z = -1j * c * dt * ks
    Rz = 1 + z + z * z / 2 + z ** 3 / 6
    discrete = np.imag(Rz ** nsteps * np.exp(1j * k * x))
    assert np.max(np.abs(phi - discrete)) < 2e-12
    err = np.max(np.abs(phi - np.sin(2 * np.pi * (x - c * T))))
    mag = g["error_order_of_magnitude"]
    assert mag / 10 < err < mag * 10, err
    # amplitude decay |R|^n - 1 dominates: about -2.6e-10
    assert abs(err - abs(abs(Rz) ** nsteps - 1)) < 2e-11
