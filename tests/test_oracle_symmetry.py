"""Symmetry boundaries of the oracle (paper Sec. "Boundary conditions": beyond each end
of a symmetry axis the fields mirror the points inside, the vector component normal to
the boundary with opposite sign).

Pins, independent of the mirror indexing in the oracle:
- a state with symmetry boundaries on N points is the restriction of a periodic state on
  2N points built by mirroring (normal momentum negated); the periodic oracle on the
  doubled box must give the same residual and the same RK3 steps;
- one-mode closed forms: a pressure wave cos(k x) on cell-centred points x = (i + 1/2) h,
  h = pi / N, which its mirror images continue smoothly;
- mass and total energy are conserved over the box (no flux through a symmetry boundary).
"""
import math

import numpy as np
import pytest

import oracle
import synth
from oracle import stencil


def extend(q, bc):
    """Mirror-extend a (5, nz, ny, nx) state across every symmetry axis (periodic on 2N)."""
    out = q.copy()
    for axis, sym in enumerate(bc):
        if not sym:
            continue
        ax = 3 - axis                      # array axis of grid axis `axis`
        mir = np.flip(out, axis=ax).copy()
        mir[1 + axis] *= -1.0              # momentum normal to the boundary
        out = np.concatenate([out, mir], axis=ax)
    return out


def restrict(q, n):
    nx, ny, nz = n
    return q[:, :nz, :ny, :nx]


def doubled(p):
    n2 = tuple(n * (2 if s else 1) for n, s in zip(p.n, p.bc))
    L2 = tuple(L * (2 if s else 1) for L, s in zip(p.length, p.bc))
    return oracle.Params(n=n2, length=L2, order=p.order, Re=p.Re, Mach=p.Mach, Pr=p.Pr, gamma=p.gamma)


CASES = [((1, 0, 0), 4), ((0, 1, 1), 4), ((1, 1, 1), 8), ((1, 1, 1), 2), ((0, 0, 1), 6)]


@pytest.mark.parametrize("bc,order", CASES)
def test_rhs_equals_periodic_on_mirrored_box(bc, order):
    n = (20, 18, 22)
    q = synth.random_conservative_state(n, seed=sum(bc) + order, mom=0.4)
    length = tuple(math.pi * (1.0 if s else 2.0) for s in bc)
    p = oracle.Params(n=n, length=length, order=order, Re=50.0, Mach=0.3, bc=bc)
    R = oracle.rhs(q, p)
    Rext = oracle.rhs(extend(q, bc), doubled(p))
    scale = np.abs(Rext).max()
    assert np.abs(R - restrict(Rext, n)).max() <= 1e-13 * scale
    # the doubled box keeps the mirror symmetry (a check of the extension itself)
    assert np.abs(extend(restrict(Rext, n), bc) - Rext).max() <= 1e-13 * scale


def test_rk3_equals_periodic_on_mirrored_box():
    bc, n, order = (1, 0, 1), (16, 16, 18), 4
    q = synth.random_conservative_state(n, seed=5, mom=0.3)
    p = oracle.Params(n=n, length=(math.pi, 2 * math.pi, math.pi), order=order, Re=100.0, Mach=0.2, bc=bc)
    a = oracle.rk3(q, p, 2e-3, 3)
    b = restrict(oracle.rk3(extend(q, bc), doubled(p), 2e-3, 3), n)
    assert np.abs(a - b).max() <= 1e-13 * np.abs(b).max()


@pytest.mark.parametrize("order", [2, 4, 8])
def test_pressure_wave_closed_form_with_symmetry(order):
    N, k, eps, M, gam = 24, 3, 1e-3, 0.2, 1.4
    h = math.pi / N
    x = (np.arange(N) + 0.5) * h
    p = oracle.Params(n=(N, 8, 8), length=(math.pi, 2 * math.pi, 2 * math.pi), order=order,
                      Re=200.0, Mach=M, Pr=0.71, gamma=gam, bc=(1, 0, 0))
    pres = 1.0 / (gam * M * M) + eps * np.cos(k * x)
    q = np.zeros((5, 8, 8, N))
    q[0] = 1.0
    q[4] = pres / (gam - 1.0)
    R = oracle.rhs(q, p)
    a = [float(v) for v in stencil.first_derivative_weights(order)]
    c0, c = stencil.second_derivative_weights(order)
    ks = 2.0 * sum(a[m] * math.sin((m + 1) * k * h) for m in range(order // 2))
    kss = -(float(c0) + 2.0 * sum(float(c[m]) * math.cos((m + 1) * k * h) for m in range(order // 2)))
    dpdx = -eps * ks / h * np.sin(k * x)
    d2p = -eps * kss / h ** 2 * np.cos(k * x)
    kappa = 1.0 / ((gam - 1.0) * M * M * 0.71 * 200.0)
    # rounding of p ~ p0 enters the differences: bound by 20 ulp(p0) times the stencil gain
    p0 = 1.0 / (gam * M * M)
    tol1 = 20 * np.finfo(float).eps * p0 / h
    tol2 = 20 * np.finfo(float).eps * p0 / h ** 2 * kappa * gam * M * M * 10
    assert np.abs(R[0]).max() < 1e-15
    assert np.abs(R[1] + dpdx).max() < tol1 < 1e-6 * np.abs(dpdx).max()
    assert np.abs(R[2]).max() < 1e-15 and np.abs(R[3]).max() < 1e-15
    assert np.abs(R[4] - kappa * gam * M * M * d2p).max() < tol2 < 1e-6 * np.abs(kappa * gam * M * M * d2p).max()


def test_mass_and_energy_conserved_with_symmetry():
    n = (18, 20, 16)
    q = synth.random_conservative_state(n, seed=9, mom=0.5)
    p = oracle.Params(n=n, length=(math.pi,) * 3, order=4, Re=30.0, Mach=0.3, bc=(1, 1, 1))
    R = oracle.rhs(q, p)
    for f in (0, 4):
        terms = np.abs(R[f]).sum()
        assert abs(R[f].sum()) <= 1e-12 * terms, f


def test_mirror_symmetric_tgv_is_a_fixed_point_of_the_extension():
    """The Taylor-Green state sampled at cell centres of [0, pi]^3 is already mirror
    symmetric: its symmetric-box residual equals the periodic 2 pi residual on the same
    points (the periodic state on 2N points is its own mirror extension)."""
    N, order = 16, 4
    h = math.pi / N
    ps = oracle.Params(n=(N,) * 3, length=(math.pi,) * 3, order=order, bc=(1, 1, 1), **synth.TGV)
    pp = oracle.Params(n=(2 * N,) * 3, length=(2 * math.pi,) * 3, order=order, **synth.TGV)
    qp = oracle.tgv_init(pp, phase=(h / 2,) * 3)
    qs = restrict(qp, (N,) * 3)
    # equal up to the rounding of sin / cos at mirrored arguments
    assert np.abs(extend(qs, (1, 1, 1)) - qp).max() <= 1e-13 * np.abs(qp).max()
    Rs = oracle.rhs(qs, ps)
    Rp = restrict(oracle.rhs(qp, pp), (N,) * 3)
    assert np.abs(Rs - Rp).max() <= 1e-11 * np.abs(Rp).max()
