"""FP64 CPU oracle of the OpenSBLI compressible Navier-Stokes hot path.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the package smoke check and the
CPU-baseline leg of the benchmark may import this package.  It shares no code
with the HIP library (``paper_1609_01277_amd``) and never imports it.

The heavy loops live in ``sbli_oracle.c`` (plain C, -O2 -ffp-contract=off,
OpenMP over z-planes).  This module compiles it with gcc on first use, loads it
with ctypes and wraps it for numpy arrays of shape (5, nz, ny, nx) in float64.
The stencil weights come from ``oracle.stencil`` (exact rationals).
"""
import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

from . import stencil

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sbli_oracle.c")
_LIB = os.path.join(_HERE, "libsbli_oracle.so")
_MAXR = 8


def build(force=False):
    """Compile the C oracle into oracle/libsbli_oracle.so (gcc, OpenMP)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
           "-std=c11", "-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


class _Grid(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int * 3), ("h", ctypes.c_double * 3), ("r", ctypes.c_int),
                ("a", ctypes.c_double * _MAXR), ("c0", ctypes.c_double),
                ("c", ctypes.c_double * _MAXR), ("Re", ctypes.c_double),
                ("Mach", ctypes.c_double), ("Pr", ctypes.c_double), ("gamma", ctypes.c_double),
                ("sym", ctypes.c_int * 3)]


RHS_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.POINTER(ctypes.c_double),
                          ctypes.POINTER(ctypes.c_double))

_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        dp = ctypes.POINTER(ctypes.c_double)
        gp = ctypes.POINTER(_Grid)
        _lib.ora_d1.argtypes = [gp, dp, ctypes.c_int, ctypes.c_int, dp]
        _lib.ora_d2.argtypes = [gp, dp, ctypes.c_int, ctypes.c_int, dp]
        _lib.ora_rhs.argtypes = [gp, dp, dp]
        _lib.ora_rk3_step.argtypes = [gp, dp, dp, ctypes.c_double, ctypes.c_int]
        _lib.ora_rk3_generic.argtypes = [ctypes.c_long, dp, dp, ctypes.c_double, ctypes.c_int,
                                         RHS_FN, ctypes.c_void_p]
        _lib.ora_tgv_init.argtypes = [gp, dp, dp]
        _lib.ora_diagnostics.argtypes = [gp, dp, dp, ctypes.POINTER(ctypes.c_long)]
        _lib.ora_num_threads.restype = ctypes.c_int
        _lib.ora_set_num_threads.argtypes = [ctypes.c_int]
    return _lib


@dataclass
class Params:
    """Problem statement: grid (N per axis, box length), order, Re, M, Pr, gamma."""
    n: tuple = (32, 32, 32)            # (nx, ny, nz)
    length: tuple = (2 * np.pi, 2 * np.pi, 2 * np.pi)
    order: int = 4
    Re: float = 1600.0
    Mach: float = 0.1
    Pr: float = 0.71
    gamma: float = 1.4
    spacing: tuple = field(default=None)  # overrides length/n when given (patch evaluation)
    bc: tuple = (0, 0, 0)              # per axis: 0 periodic, 1 symmetry boundaries

    def h(self):
        if self.spacing is not None:
            return tuple(float(s) for s in self.spacing)
        return tuple(float(L) / int(n) for L, n in zip(self.length, self.n))


def _grid(p: Params):
    g = _Grid()
    for i in range(3):
        g.n[i] = int(p.n[i])
    for i, hh in enumerate(p.h()):
        g.h[i] = hh
    r = p.order // 2
    if r < 1 or r > _MAXR:
        raise ValueError("order out of range")
    g.r = r
    a = stencil.first_derivative_weights(p.order)
    c0, c = stencil.second_derivative_weights(p.order)
    for m in range(r):
        g.a[m] = float(a[m])
        g.c[m] = float(c[m])
    g.c0 = float(c0)
    g.Re, g.Mach, g.Pr, g.gamma = float(p.Re), float(p.Mach), float(p.Pr), float(p.gamma)
    for i in range(3):
        if p.bc[i] not in (0, 1):
            raise ValueError("bc must be 0 (periodic) or 1 (symmetry) per axis")
        g.sym[i] = int(p.bc[i])
    return g


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _state(q, p):
    q = np.ascontiguousarray(q, dtype=np.float64)
    nx, ny, nz = p.n
    if q.shape != (5, nz, ny, nx):
        raise ValueError("state must have shape (5, nz, ny, nx) = %r, got %r" % ((5, nz, ny, nx), q.shape))
    return q


def d1(f, axis, p: Params, parity=1):
    """Order-p central first derivative of a (nz, ny, nx) array along axis 0=x, 1=y, 2=z.
    parity (+1 / -1): how f continues beyond a symmetry boundary on that axis."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    out = np.empty_like(f)
    g = _grid(p)
    lib().ora_d1(ctypes.byref(g), _dp(f), int(axis), int(parity), _dp(out))
    return out


def d2(f, axis, p: Params, parity=1):
    """Order-p central second derivative along axis 0=x, 1=y, 2=z (parity as in d1)."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    out = np.empty_like(f)
    g = _grid(p)
    lib().ora_d2(ctypes.byref(g), _dp(f), int(axis), int(parity), _dp(out))
    return out


def tgv_init(p: Params, phase=(0.0, 0.0, 0.0)):
    """Taylor-Green initial state, shape (5, nz, ny, nx)."""
    nx, ny, nz = p.n
    q = np.empty((5, nz, ny, nx), dtype=np.float64)
    ph = np.asarray(phase, dtype=np.float64)
    g = _grid(p)
    lib().ora_tgv_init(ctypes.byref(g), _dp(q), _dp(ph))
    return q


def rhs(q, p: Params):
    """Residual R = dq/dt of the compressible Navier-Stokes equations."""
    q = _state(q, p)
    out = np.empty_like(q)
    g = _grid(p)
    lib().ora_rhs(ctypes.byref(g), _dp(q), _dp(out))
    return out


def rk3(q, p: Params, dt, nsteps=1):
    """nsteps low-storage RK3 steps; returns the new state (input untouched)."""
    q = _state(q, p).copy()
    dq = np.zeros_like(q)
    g = _grid(p)
    lib().ora_rk3_step(ctypes.byref(g), _dp(q), _dp(dq), float(dt), int(nsteps))
    return q


def rk3_generic(y, dt, nsteps, f):
    """The same RK3 scheme on an arbitrary ODE system y' = f(y) (f: ndarray -> ndarray)."""
    y = np.ascontiguousarray(y, dtype=np.float64).copy()
    n = y.size
    dq = np.zeros_like(y)

    def cb(_ctx, yp, Rp):
        yy = np.ctypeslib.as_array(yp, shape=(n,))
        RR = np.ctypeslib.as_array(Rp, shape=(n,))
        RR[:] = f(yy.copy())

    fn = RHS_FN(cb)
    lib().ora_rk3_generic(n, _dp(y), _dp(dq), float(dt), int(nsteps), fn, None)
    return y


def diagnostics(q, p: Params):
    """(E_k, enstrophy, <rho>, <rho u>, <rho v>, <rho w>, <rho E>), flags (nonfinite, rho<=0, p<=0)."""
    q = _state(q, p)
    out = np.zeros(7, dtype=np.float64)
    flags = (ctypes.c_long * 3)()
    g = _grid(p)
    lib().ora_diagnostics(ctypes.byref(g), _dp(q), _dp(out), flags)
    return out, (flags[0], flags[1], flags[2])


def rk3_at_points(q, p: Params, dt, points, nsteps=1):
    """One-by-one oracle values of `nsteps` RK3 steps at the given (x, y, z) points.

    Each RK3 stage reads the state within 2r points along the axes, so after
    `nsteps` steps a point depends only on the state inside a cube of half-width
    6 r nsteps.  For each point this copies that cube (periodic wrap), treats it
    as a periodic box with the original spacing, runs the ordinary whole-array
    oracle on it and keeps the centre value, which is then the same arithmetic
    as on the full grid: the wrapped edges of the copy never reach the centre.
    Returns an array (len(points), 5).
    """
    if any(p.bc):
        raise ValueError("patch evaluation assumes periodic axes")
    q = _state(q, p)
    nx, ny, nz = p.n
    r = p.order // 2
    w = 6 * r * nsteps
    size = 2 * w + 1
    sub = Params(n=(size, size, size), order=p.order, Re=p.Re, Mach=p.Mach, Pr=p.Pr,
                 gamma=p.gamma, spacing=p.h())
    out = np.empty((len(points), 5))
    for n_, (x, y, z) in enumerate(points):
        ix = np.arange(x - w, x + w + 1) % nx
        iy = np.arange(y - w, y + w + 1) % ny
        iz = np.arange(z - w, z + w + 1) % nz
        patch = q[:, iz][:, :, iy][:, :, :, ix]
        res = rk3(patch, sub, dt, nsteps)
        out[n_] = res[:, w, w, w]
    return out


def rhs_at_points(q, p: Params, points):
    """One-by-one oracle residual at the given (x, y, z) points (patch of half-width 2r)."""
    if any(p.bc):
        raise ValueError("patch evaluation assumes periodic axes")
    q = _state(q, p)
    nx, ny, nz = p.n
    r = p.order // 2
    w = 2 * r
    size = 2 * w + 1
    sub = Params(n=(size, size, size), order=p.order, Re=p.Re, Mach=p.Mach, Pr=p.Pr,
                 gamma=p.gamma, spacing=p.h())
    out = np.empty((len(points), 5))
    for n_, (x, y, z) in enumerate(points):
        ix = np.arange(x - w, x + w + 1) % nx
        iy = np.arange(y - w, y + w + 1) % ny
        iz = np.arange(z - w, z + w + 1) % nz
        patch = q[:, iz][:, :, iy][:, :, :, ix]
        out[n_] = rhs(patch, sub)[:, w, w, w]
    return out


def num_threads():
    return lib().ora_num_threads()


def set_num_threads(n):
    lib().ora_set_num_threads(int(n))
