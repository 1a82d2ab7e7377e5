"""Pins of the oracle's Taylor-Green initial state, diagnostics and time integration
(paper Sec. "3D Taylor-Green vortex": initial conditions, kinetic-energy and enstrophy
integrals)."""
import json
import math
import os

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
G = json.load(open(os.path.join(GOLDEN, "tgv_initial.json")))


def params(n, order=4):
    if isinstance(n, int):
        n = (n, n, n)
    return oracle.Params(n=n, order=order, Re=G["Re"], Mach=G["Mach"], Pr=G["Pr"], gamma=G["gamma"])


def s_mod(order, n):
    # modified wavenumber of the order-p first derivative at k = 1 (textbook weights)
    r = order // 2
    h = 2 * np.pi / n
    a = [(-1) ** (m + 1) * math.factorial(r) ** 2 / (m * math.factorial(r - m) * math.factorial(r + m))
         for m in range(1, r + 1)]
    return 2 / h * sum(a[m - 1] * math.sin(m * h) for m in range(1, r + 1))


@pytest.mark.parametrize("n,order", [(32, 4), (24, 4), ((27, 30, 33), 4), (32, 8), (64, 4)])
def test_initial_diagnostics_closed_form(oracle_mod, n, order):
    p = params(n, order)
    q = oracle.tgv_init(p)
    d, flags = oracle.diagnostics(q, p)
    assert flags == (0, 0, 0)
    g, M = G["gamma"], G["Mach"]
    assert abs(d[0] - 1 / 8) < 1e-15
    assert abs(d[2] - 1.0) < 1e-15
    assert max(abs(d[3]), abs(d[4]), abs(d[5])) < 1e-16
    assert abs(d[6] - (1 / (g * (g - 1) * M * M) + 1 / 8)) < 1e-12
    nn = n if isinstance(n, int) else None
    if nn is not None:
        assert abs(d[1] - 3 / 8 * s_mod(order, nn) ** 2) < 1e-14


def test_initial_enstrophy_values_at_32_and_64(oracle_mod):
    # eps_h(0) = (3/8) s^2 for the 4th-order stencil at 32^3 and 64^3
    for n, expect in ((32, 0.374963012455195), (64, 0.374997680253154)):
        p = params(n, 4)
        d, _ = oracle.diagnostics(oracle.tgv_init(p), p)
        assert abs(d[1] - expect) < 1e-14


def test_initial_pointwise_fields(oracle_mod):
    n = 16
    p = params(n)
    q = oracle.tgv_init(p)
    h = 2 * np.pi / n
    x = np.arange(n) * h
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    g, M = G["gamma"], G["Mach"]
    u = np.sin(X) * np.cos(Y) * np.cos(Z)
    v = -np.cos(X) * np.sin(Y) * np.cos(Z)
    pr = 1 / (g * M * M) + (np.cos(2 * X) + np.cos(2 * Y)) * (np.cos(2 * Z) + 2) / 16
    assert np.abs(q[0] - 1).max() == 0
    assert np.abs(q[1] - u).max() < 1e-15 and np.abs(q[2] - v).max() < 1e-15
    assert np.abs(q[3]).max() == 0
    assert np.abs(q[4] - (pr / (g - 1) + 0.5 * (u * u + v * v))).max() < 1e-12


def test_diagnostic_flags(oracle_mod):
    n = 16
    p = params(n)
    q = oracle.tgv_init(p)
    q[2, 3, 4, 5] = np.nan
    q[0, 1, 1, 1] = -1.0
    q[4, 7, 7, 7] = 0.0      # p < 0 there
    _, flags = oracle.diagnostics(q, p)
    assert flags[0] == 1
    assert flags[1] == 1
    assert flags[2] >= 1


def test_temporal_self_convergence_third_order(oracle_mod):
    # TGV 32^3, fixed spatial operator: halving dt divides the time error by ~8.  The
    # steps keep the acoustic z = c k* dt below ~0.2 so the leading error term dominates.
    n = 32
    p = params(n)
    q0 = oracle.tgv_init(p)
    T = 0.05
    sols = []
    for nsteps in (20, 40, 80, 160):
        sols.append(oracle.rk3(q0, p, T / nsteps, nsteps))
    e = [np.abs(sols[i] - sols[i + 1]).max() for i in range(3)]
    assert abs(e[0] / e[1] - 8) < 0.3 and abs(e[1] / e[2] - 8) < 0.3, e


def test_energy_decay_rate_matches_enstrophy(oracle_mod):
    # Physical sanity (approximate): dE_k/dt ~ -2 eps / Re at t = 0 for M = 0.1.
    n = 32
    p = params(n)
    q0 = oracle.tgv_init(p)
    d0, _ = oracle.diagnostics(q0, p)
    dt = 1e-3
    d1, _ = oracle.diagnostics(oracle.rk3(q0, p, dt, 1), p)
    rate = (d1[0] - d0[0]) / dt
    expect = -2 * d0[1] / G["Re"]
    assert abs(rate / expect - 1) < 0.05, (rate, expect)


def test_conservation_over_steps(oracle_mod):
    n = 24
    p = params(n, 8)
    q0 = oracle.tgv_init(p)
    d0, _ = oracle.diagnostics(q0, p)
    d1, _ = oracle.diagnostics(oracle.rk3(q0, p, 5e-3, 5), p)
    for f in range(2, 7):
        assert abs(d1[f] - d0[f]) < 1e-13 * max(1.0, abs(d0[f]))


def test_patch_evaluation_equals_full_grid(oracle_mod):
    # The one-by-one evaluator (a cube of half-width 6 r around a point) reproduces the
    # whole-grid oracle bitwise.
    n = 30
    p = params(n, 4)
    q0 = oracle.tgv_init(p) + 0.01 * np.random.default_rng(3).standard_normal((5, n, n, n))
    full = oracle.rk3(q0, p, 2e-3, 1)
    pts = [(0, 0, 0), (29, 1, 17), (5, 28, 13)]
    loc = oracle.rk3_at_points(q0, p, 2e-3, pts)
    for (x, y, z), v in zip(pts, loc):
        assert np.array_equal(full[:, z, y, x], v)
    R = oracle.rhs(q0, p)
    locR = oracle.rhs_at_points(q0, p, pts)
    for (x, y, z), v in zip(pts, locR):
        assert np.array_equal(R[:, z, y, x], v)
