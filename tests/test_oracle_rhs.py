"""Pins of the oracle's Navier-Stokes residual (paper Sec. "3D Taylor-Green vortex":
eq. mass, momentum, energy, stress tensor, heat flux, eq. eos, total energy and the
skew-symmetric convective form).

Each test fixes something the paper or the mathematics determines without the
oracle: exact discrete conservation, closed forms on one-mode states (computed
with the textbook stencil weights), convergence at the design order to the
symbolically differentiated conservation laws, and symmetries.
"""
import math

import numpy as np
import pytest

import oracle
import synth

GAMMA, MACH, PR, RE = 1.4, 0.1, 0.71, 1600.0


def ks(order, k, h):
    """Modified wavenumber of the order-p first derivative for mode k (textbook weights)."""
    r = order // 2
    a = [(-1) ** (m + 1) * math.factorial(r) ** 2 / (m * math.factorial(r - m) * math.factorial(r + m))
         for m in range(1, r + 1)]
    return 2 / h * sum(a[m - 1] * math.sin(m * k * h) for m in range(1, r + 1))


def kss(order, k, h):
    """Modified wavenumber of the order-p second derivative: D2 e^{ikx} = -kss e^{ikx}."""
    r = order // 2
    a = [(-1) ** (m + 1) * math.factorial(r) ** 2 / (m * math.factorial(r - m) * math.factorial(r + m))
         for m in range(1, r + 1)]
    c = [2 * a[m - 1] / m for m in range(1, r + 1)]
    c0 = -2 * sum(c)
    return (-c0 - 2 * sum(c[m - 1] * math.cos(m * k * h) for m in range(1, r + 1))) / h ** 2


def coords(n):
    h = 2 * np.pi / n
    x = np.arange(n) * h
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    return (X, Y, Z), h


def cons(rho, u, p):
    """Conservative state from primitives (test-side helper; total energy definition)."""
    rE = p / (GAMMA - 1) + 0.5 * rho * (u[0] ** 2 + u[1] ** 2 + u[2] ** 2)
    return np.stack([rho, rho * u[0], rho * u[1], rho * u[2], rE])


def params(n, order, Re=RE, Mach=MACH):
    return oracle.Params(n=(n, n, n), order=order, Re=Re, Mach=Mach, Pr=PR, gamma=GAMMA)


@pytest.mark.parametrize("order", [2, 4, 8])
@pytest.mark.parametrize("n", [(17, 18, 19), (20, 20, 20)])
def test_discrete_conservation_random_state(oracle_mod, order, n):
    # D is an antisymmetric circulant and D2 a zero-sum circulant: every term of the
    # skew-symmetric residual sums to zero over the periodic box, for ANY state.
    q = synth.random_conservative_state(n, seed=11 + order)
    p = oracle.Params(n=n, order=order)
    R = oracle.rhs(q, p)
    P = np.prod(n)
    for f in range(5):
        tot = R[f].sum()
        scale = np.abs(R[f]).sum() + P
        assert abs(tot) < 1e-12 * scale, (f, tot, scale)
    # and the residual is not trivially small
    assert np.abs(R).max() > 1.0


@pytest.mark.parametrize("order", [4, 8])
@pytest.mark.parametrize("axis", [0, 1, 2])
def test_pressure_wave_closed_form(oracle_mod, order, axis):
    # rho = 1, u = 0, p = p0 + e cos(kx):  R_rho = 0, R_m = -D p (along the axis only),
    # R_E = kappa * D2 T with T = gamma M^2 p  (heat flux with positive diffusivity).
    n, k, eps = 24, 2, 1e-3
    (X, Y, Z), h = coords(n)
    xa = (X, Y, Z)[axis]
    p0 = 1 / (GAMMA * MACH ** 2)
    pr = p0 + eps * np.cos(k * xa)
    q = cons(np.ones_like(X), [0 * X, 0 * X, 0 * X], pr)
    R = oracle.rhs(q, params(n, order))
    kappa = 1 / ((GAMMA - 1) * MACH ** 2 * PR * RE)
    assert np.abs(R[0]).max() < 1e-13
    for i in range(3):
        exp = eps * ks(order, k, h) * np.sin(k * xa) if i == axis else 0 * X
        assert np.abs(R[1 + i] - exp).max() < 1e-11
    expE = kappa * GAMMA * MACH ** 2 * (-kss(order, k, h)) * eps * np.cos(k * xa)
    assert np.abs(R[4] - expE).max() < 1e-11


@pytest.mark.parametrize("order", [4, 8])
@pytest.mark.parametrize("axis", [0, 2])
def test_isothermal_density_wave_in_uniform_flow(oracle_mod, order, axis):
    # rho = 1 + e cos(kx), u = U e_axis, p = p0 rho (so T is uniform):
    #   R_rho = -U D rho,  R_m[axis] = -(U^2 + p0) D rho,
    #   R_E = -U (p0/(gamma-1) + U^2/2 + p0) D rho,   with D rho = -e k* sin(kx).
    n, k, eps, U = 24, 3, 1e-2, 0.7
    (X, Y, Z), h = coords(n)
    xa = (X, Y, Z)[axis]
    p0 = 1 / (GAMMA * MACH ** 2)
    rho = 1 + eps * np.cos(k * xa)
    u = [0 * X, 0 * X, 0 * X]
    u[axis] = U + 0 * X
    q = cons(rho, u, p0 * rho)
    R = oracle.rhs(q, params(n, order))
    Drho = -eps * ks(order, k, h) * np.sin(k * xa)
    tol = 1e-10
    assert np.abs(R[0] - (-U * Drho)).max() < tol
    for i in range(3):
        exp = -(U * U + p0) * Drho if i == axis else 0 * X
        assert np.abs(R[1 + i] - exp).max() < tol
    et = p0 / (GAMMA - 1) + 0.5 * U * U
    assert np.abs(R[4] - (-U * (et + p0) * Drho)).max() < 1e-9


@pytest.mark.parametrize("order", [4, 8])
def test_shear_wave_viscous_terms(oracle_mod, order):
    # rho = 1, u = (0, e sin kx, 0), p = p0:
    #   R_rhov = (1/Re) D2_x v = -(1/Re) k** e sin kx
    #   R_rhoE = D_x(v tau_yx) = (1/Re) D_x(v D_x v) = (1/Re) e^2/2 k*(k) k*(2k) cos 2kx
    n, k, eps = 24, 2, 0.1
    (X, Y, Z), h = coords(n)
    p0 = 1 / (GAMMA * MACH ** 2)
    q = cons(np.ones_like(X), [0 * X, eps * np.sin(k * X), 0 * X], p0 + 0 * X)
    R = oracle.rhs(q, params(n, order))
    assert np.abs(R[0]).max() < 1e-13
    assert np.abs(R[1]).max() < 1e-12 and np.abs(R[3]).max() < 1e-12
    assert np.abs(R[2] - (-(1 / RE) * kss(order, k, h) * eps * np.sin(k * X))).max() < 1e-12
    expE = (1 / RE) * 0.5 * eps ** 2 * ks(order, k, h) * ks(order, 2 * k, h) * np.cos(2 * k * X)
    assert np.abs(R[4] - expE).max() < 1e-11


@pytest.mark.parametrize("order", [4, 8])
def test_compressive_wave_momentum(oracle_mod, order):
    # rho = 1, u = (e sin kx, 0, 0), p = p0:
    #   R_rho = -e k* cos kx
    #   R_rhou = -e^2/4 [k*(2k) + 2 k*(k)] sin 2kx - (4/(3 Re)) k** e sin kx
    n, k, eps = 24, 2, 0.2
    (X, Y, Z), h = coords(n)
    p0 = 1 / (GAMMA * MACH ** 2)
    q = cons(np.ones_like(X), [eps * np.sin(k * X), 0 * X, 0 * X], p0 + 0 * X)
    R = oracle.rhs(q, params(n, order))
    assert np.abs(R[0] - (-eps * ks(order, k, h) * np.cos(k * X))).max() < 1e-12
    exp = (-0.25 * eps ** 2 * (ks(order, 2 * k, h) + 2 * ks(order, k, h)) * np.sin(2 * k * X)
           - 4 / (3 * RE) * kss(order, k, h) * eps * np.sin(k * X))
    assert np.abs(R[1] - exp).max() < 1e-12


@pytest.mark.parametrize("order", [4, 8])
def test_mixed_nested_second_derivative(oracle_mod, order):
    # rho = 1, u = (0, e sin kx sin ly, 0), p = p0: the only contribution to R_rhou is the
    # nested grad-div part (1/(3 Re)) D_x(D_y v) = (1/(3 Re)) e k*(k) l*(l) cos kx cos ly.
    n, k, l, eps = 24, 2, 3, 0.1
    (X, Y, Z), h = coords(n)
    p0 = 1 / (GAMMA * MACH ** 2)
    q = cons(np.ones_like(X), [0 * X, eps * np.sin(k * X) * np.sin(l * Y), 0 * X], p0 + 0 * X)
    R = oracle.rhs(q, params(n, order))
    exp = eps * ks(order, k, h) * ks(order, l, h) * np.cos(k * X) * np.cos(l * Y) / (3 * RE)
    assert np.abs(R[1] - exp).max() < 1e-12
    assert np.abs(R[0] - (-eps * ks(order, l, h) * np.sin(k * X) * np.cos(l * Y))).max() < 1e-12


def _mms_exact(n, Re, Mach):
    """Manufactured smooth state and its exact continuous residual, by sympy, from the
    conservation laws in divergence form (eq. mass, momentum, energy; mu = 1)."""
    import sympy as sp
    x, y, z = sp.symbols("x y z")
    X3 = (x, y, z)
    g, M, Pr = sp.Rational(7, 5), sp.nsimplify(Mach), sp.Rational(71, 100)
    Re_s = sp.nsimplify(Re)
    rho = 1 + sp.Rational(1, 5) * sp.sin(x + 2 * y) * sp.cos(z)
    u = [sp.Rational(1, 2) * sp.sin(x) * sp.cos(2 * y + z),
         -sp.Rational(1, 3) * sp.cos(2 * x) * sp.sin(y - z),
         sp.Rational(1, 4) * sp.sin(x + y) * sp.cos(2 * z)]
    p = 1 / (g * M ** 2) + sp.Rational(1, 5) * sp.cos(x - y) * sp.sin(z + x)
    rE = p / (g - 1) + rho * sum(ui ** 2 for ui in u) / 2
    T = g * M ** 2 * p / rho
    kappa = 1 / ((g - 1) * M ** 2 * Pr * Re_s)
    div = sum(sp.diff(u[k], X3[k]) for k in range(3))
    tau = [[(sp.diff(u[i], X3[j]) + sp.diff(u[j], X3[i]) - (sp.Rational(2, 3) * div if i == j else 0)) / Re_s
            for j in range(3)] for i in range(3)]
    R = [-sum(sp.diff(rho * u[j], X3[j]) for j in range(3))]
    for i in range(3):
        R.append(-sum(sp.diff(rho * u[i] * u[j] + (p if i == j else 0) - tau[i][j], X3[j]) for j in range(3)))
    R.append(-sum(sp.diff((rE + p) * u[j] - kappa * sp.diff(T, X3[j])
                          - sum(u[i] * tau[i][j] for i in range(3)), X3[j]) for j in range(3)))
    fq = sp.lambdify(X3, [rho, rho * u[0], rho * u[1], rho * u[2], rE], "numpy")
    fR = sp.lambdify(X3, R, "numpy")
    (Xg, Yg, Zg), h = coords(n)
    q = np.stack([np.broadcast_to(np.asarray(v, dtype=float), Xg.shape) for v in fq(Xg, Yg, Zg)])
    Rex = np.stack([np.broadcast_to(np.asarray(v, dtype=float), Xg.shape) for v in fR(Xg, Yg, Zg)])
    return q, Rex


@pytest.mark.parametrize("order", [4, 8])
def test_manufactured_solution_spatial_order(oracle_mod, order):
    # The discrete skew-symmetric residual converges to the exact residual of the
    # conservation laws at the design order; any dropped term, wrong sign, wrong
    # coefficient or transposed index stalls the convergence.  Re and M are chosen so
    # the viscous and heat-flux terms are O(1).
    Re, Mach = 5.0, 0.5
    sizes = (32, 64) if order == 4 else (32, 48)
    errs = []
    for n in sizes:
        q, Rex = _mms_exact(n, Re, Mach)
        R = oracle.rhs(q, params(n, order, Re=Re, Mach=Mach))
        errs.append([np.abs(R[f] - Rex[f]).max() / np.abs(Rex[f]).max() for f in range(5)])
    for f in range(5):
        slope = math.log(errs[0][f] / errs[1][f]) / math.log(sizes[1] / sizes[0])
        assert abs(slope - order) < (0.3 if order == 4 else 1.0), (order, f, errs)
        assert errs[1][f] < 1e-3


@pytest.mark.parametrize("order", [4, 8])
def test_roll_equivariance_bitwise(oracle_mod, order):
    n = 18
    q = synth.random_conservative_state(n, seed=5)
    p = params(n, order)
    R = oracle.rhs(q, p)
    shift = (3, -5, 7)
    qr = np.roll(q, shift, axis=(3, 2, 1))
    Rr = oracle.rhs(qr, p)
    assert np.array_equal(Rr, np.roll(R, shift, axis=(3, 2, 1)))


@pytest.mark.parametrize("order", [4, 8])
def test_axis_permutation_equivariance(oracle_mod, order):
    # swapping x and y (and the u, v components) commutes with the residual
    n = 18
    q = synth.random_conservative_state(n, seed=9)
    p = params(n, order)
    R = oracle.rhs(q, p)
    qs = q[[0, 2, 1, 3, 4]].transpose(0, 1, 3, 2).copy()
    Rs = oracle.rhs(qs, p)
    Rback = Rs[[0, 2, 1, 3, 4]].transpose(0, 1, 3, 2)
    for f in range(5):
        assert np.abs(Rback[f] - R[f]).max() <= 1e-12 * (np.abs(R[f]).max() + 1)


def test_tgv_reflection_parities(oracle_mod):
    # Taylor-Green symmetry x -> -x: rho, rho v, rho w, rho E even; rho u odd (the residual too).
    n = 24
    p = params(n, 4)
    q = oracle.tgv_init(p)
    R = oracle.rhs(q, p)
    ref = lambda a: np.roll(a[..., ::-1], 1, axis=-1)  # noqa: E731  index i -> -i mod n
    for f, sign in zip(range(5), (1, -1, 1, 1, 1)):
        assert np.abs(ref(q[f]) - sign * q[f]).max() < 1e-13
        assert np.abs(ref(R[f]) - sign * R[f]).max() < 1e-11
