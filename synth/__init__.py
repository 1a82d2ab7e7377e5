"""Seeded synthetic inputs shared by the oracle side and the GPU side of tests and benchmarks.

This module holds random draws only: no step of the solver's arithmetic (no
equation of state, no derivative, no time stepping).  Both sides receive the
same arrays or parameters from here.
"""
import math

import numpy as np

# Taylor-Green parameters (paper Sec. "3D Taylor-Green vortex").
TGV = dict(Re=1600.0, Mach=0.1, Pr=0.71, gamma=1.4)
# Time step of the 64^3 run, halved at each doubling of the grid.
DT64 = 3.385e-3


def tgv_dt(n):
    """Time step for an n^3 Taylor-Green grid: 3.385e-3 at 64^3, halved per doubling."""
    return DT64 * 64.0 / n


def random_conservative_state(n, seed, rho=(0.9, 1.1), mom=1.0, energy=(178.0, 180.0)):
    """Random conservative state (5, nz, ny, nx), float64, from a seed.

    rho ~ U(rho), rho*u_i ~ U(-mom, mom), rho*E ~ U(energy).  With the default
    ranges every point has rho > 0 and a positive pressure for gamma = 1.4.
    """
    if isinstance(n, int):
        n = (n, n, n)
    nx, ny, nz = n
    rng = np.random.default_rng(seed)
    q = np.empty((5, nz, ny, nx))
    q[0] = rng.uniform(rho[0], rho[1], (nz, ny, nx))
    q[1:4] = rng.uniform(-mom, mom, (3, nz, ny, nx))
    q[4] = rng.uniform(energy[0], energy[1], (nz, ny, nx))
    return q


def smooth_random_perturbation(n, seed, amplitude=0.05, kmax=3):
    """Sum of random low-wavenumber Fourier modes on an n^3 periodic grid, shape (5, n, n, n).

    Used to perturb a Taylor-Green state into a generic smooth state.  Each field
    gets its own random amplitudes and phases for integer wavevectors |k_i| <= kmax.
    """
    rng = np.random.default_rng(seed)
    x = 2 * np.pi * np.arange(n) / n
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    out = np.zeros((5, n, n, n))
    for f in range(5):
        for _ in range(6):
            k = rng.integers(-kmax, kmax + 1, size=3)
            a = rng.uniform(-amplitude, amplitude)
            ph = rng.uniform(0, 2 * np.pi)
            out[f] += a * np.cos(k[0] * X + k[1] * Y + k[2] * Z + ph)
    return out


def batch_instances(count=64, seed=1609, sizes=(32, 48, 64, 96, 128), re=(400.0, 3200.0),
                    mach=(0.1, 0.4), courant=0.379273, pr=0.71, gamma=1.4):
    """Ensemble of Taylor-Green instances from a seed.

    N uniform over `sizes`, Re ~ U(re), M ~ U(mach), phase ~ U[0, 2 pi)^3.  The
    time step keeps the acoustic Courant number of the paper's 64^3 run
    (dt = 3.385e-3 with |u| + c = 1 + 1/M = 11):  dt = courant * h / (1 + 1/M).
    Returns a list of dicts with keys n, Re, Mach, Pr, gamma, dt, phase.
    """
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        n = int(rng.choice(sizes))
        Re = float(rng.uniform(*re))
        M = float(rng.uniform(*mach))
        phase = [float(v) for v in rng.uniform(0.0, 2 * math.pi, 3)]
        h = 2 * math.pi / n
        dt = courant * h / (1.0 + 1.0 / M)
        out.append(dict(n=n, Re=Re, Mach=M, Pr=pr, gamma=gamma, dt=dt, phase=phase))
    return out


def closure_init_params(seed, channels=(5, 32, 32, 5)):
    """Initial closure-network parameters from a seed, flat float32 vector.

    Per layer W[out][in][3][3][3] ~ U(-b, b) with b = sqrt(6 / (27 in)) (He-uniform
    for a 3x3x3 kernel), then zero biases; layers back to back.
    """
    rng = np.random.default_rng(seed)
    parts = []
    for ci, co in zip(channels[:-1], channels[1:]):
        bound = math.sqrt(6.0 / (ci * 27))
        parts.append(rng.uniform(-bound, bound, co * ci * 27))
        parts.append(np.zeros(co))
    return np.concatenate(parts).astype(np.float32)
