"""Pins of the oracle's central-difference operators (paper Sec. "Discretisation schemes").

The oracle solves a Vandermonde system for the weights; these tests hold it to
(1) the textbook closed form of the central weights, (2) exactness on
polynomials by brute force in rationals, and (3) the C stencils' action on
Fourier modes (modified wavenumbers) and their convergence order.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import stencil


def closed_form_a(r):
    # a_m = (-1)^(m+1) (r!)^2 / (m (r-m)! (r+m)!)   (e.g. Fornberg 1988, central case)
    return [Fraction((-1) ** (m + 1) * math.factorial(r) ** 2,
                     m * math.factorial(r - m) * math.factorial(r + m)) for m in range(1, r + 1)]


@pytest.mark.parametrize("order", [2, 4, 6, 8, 10, 12])
def test_weights_match_closed_form(order):
    r = order // 2
    a = stencil.first_derivative_weights(order)
    assert a == closed_form_a(r)
    c0, c = stencil.second_derivative_weights(order)
    assert c == [2 * am / m for m, am in enumerate(closed_form_a(r), start=1)]
    assert c0 == -2 * sum(c)


def test_weights_printed_values():
    # The familiar 4th- and 8th-order tables.
    assert stencil.first_derivative_weights(4) == [Fraction(2, 3), Fraction(-1, 12)]
    assert stencil.second_derivative_weights(4) == (Fraction(-5, 2), [Fraction(4, 3), Fraction(-1, 12)])
    assert stencil.first_derivative_weights(8) == [Fraction(4, 5), Fraction(-1, 5), Fraction(4, 105),
                                                    Fraction(-1, 280)]
    c0, c = stencil.second_derivative_weights(8)
    assert c0 == Fraction(-205, 72)
    assert c == [Fraction(8, 5), Fraction(-1, 5), Fraction(8, 315), Fraction(-1, 560)]


@pytest.mark.parametrize("order", [2, 4, 6, 8])
def test_polynomial_exactness_bruteforce(order):
    # Apply the stencil to x^q sampled at integer offsets around a non-zero point x0.
    r = order // 2
    a = stencil.first_derivative_weights(order)
    c0, c = stencil.second_derivative_weights(order)
    x0 = Fraction(3, 7)
    for q in range(0, order + 2):
        f = lambda x: x ** q  # noqa: E731
        d1 = sum(a[m - 1] * (f(x0 + m) - f(x0 - m)) for m in range(1, r + 1))
        d2 = c0 * f(x0) + sum(c[m - 1] * (f(x0 + m) + f(x0 - m)) for m in range(1, r + 1))
        ex1 = q * x0 ** (q - 1) if q >= 1 else 0
        ex2 = q * (q - 1) * x0 ** (q - 2) if q >= 2 else 0
        if q <= order:
            assert d1 == ex1, (order, q)
        if q <= order + 1:
            assert d2 == ex2, (order, q)
    # ...and not beyond: degree order+1 breaks the first derivative.
    q = order + 1
    d1 = sum(a[m - 1] * ((x0 + m) ** q - (x0 - m) ** q) for m in range(1, r + 1))
    assert d1 != q * x0 ** (q - 1)


def _grid(n, order, axis_len=2 * np.pi):
    return oracle.Params(n=n, order=order, length=(axis_len,) * 3)


@pytest.mark.parametrize("order", [2, 4, 6, 8])
@pytest.mark.parametrize("axis", [0, 1, 2])
def test_c_stencils_on_fourier_modes(oracle_mod, order, axis):
    # D e^{ikx} = i k* e^{ikx},  k* = (2/h) sum a_m sin(m k h)
    # D2 e^{ikx} = -k** e^{ikx}, k** = (1/h^2)(-c0 - 2 sum c_m cos(m k h))
    n = [12, 10, 14]
    n[axis] = 24
    p = _grid(tuple(n), order)
    h = 2 * np.pi / 24
    x = np.arange(24) * h
    r = order // 2
    a = closed_form_a(r)
    ca = [2 * float(am) / m for m, am in enumerate(a, start=1)]
    c0 = -2 * sum(ca)
    for k in (1, 3, 5):
        ks = 2 / h * sum(float(a[m - 1]) * math.sin(m * k * h) for m in range(1, r + 1))
        kss = (-c0 - 2 * sum(ca[m - 1] * math.cos(m * k * h) for m in range(1, r + 1))) / h ** 2
        shape = [1, 1, 1]
        shape[2 - axis] = 24
        f = np.broadcast_to(np.sin(k * x + 0.3).reshape(shape), (n[2], n[1], n[0])).copy()
        df = oracle.d1(f, axis, p)
        d2f = oracle.d2(f, axis, p)
        exp1 = np.broadcast_to((ks * np.cos(k * x + 0.3)).reshape(shape), f.shape)
        exp2 = np.broadcast_to((-kss * np.sin(k * x + 0.3)).reshape(shape), f.shape)
        assert np.max(np.abs(df - exp1)) < 1e-12 * max(1.0, k * k)
        assert np.max(np.abs(d2f - exp2)) < 1e-11 * max(1.0, k ** 3)


@pytest.mark.parametrize("order", [2, 4, 6, 8])
def test_convergence_order(oracle_mod, order):
    # Error of D sin and D2 sin against the exact derivatives falls as h^order.
    errs1, errs2 = [], []
    for n in (16, 32, 64):
        p = _grid((n, 17, 17), order)
        x = np.arange(n) * 2 * np.pi / n
        f = np.broadcast_to(np.sin(x), (17, 17, n)).copy()
        errs1.append(np.max(np.abs(oracle.d1(f, 0, p) - np.cos(x))))
        errs2.append(np.max(np.abs(oracle.d2(f, 0, p) + np.sin(x))))
    for e in (errs1, errs2):
        slope = math.log2(e[0] / e[1])
        if e[1] > 1e-12:
            assert abs(slope - order) < 0.15, (order, e)
