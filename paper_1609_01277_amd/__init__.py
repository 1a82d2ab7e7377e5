"""MI355X (gfx950) compressible Navier-Stokes hot path after OpenSBLI (arXiv:1609.01277).

The solver lives in libsbli.so (hand-written HIP kernels behind a C ABI,
include/sbli.h).  This package is the thin Python side: ctypes marshalling
(`_lib`, functions named like the C entry points) and a `Solver` convenience
class that uses PyTorch only to allocate device memory and to pick the stream.
"""
import math

from . import _lib, tuning
from ._lib import (SBLI_ERR_ALLOC, SBLI_ERR_ARG, SBLI_ERR_HIP, SBLI_ERR_NONFINITE,  # noqa: F401
                   SBLI_ERR_UNSUPPORTED, SBLI_F32, SBLI_F64, SBLI_OK, SbliError, sbli_destroy,
                   sbli_diagnostics, sbli_init, sbli_last_error, sbli_params, sbli_rhs,
                   sbli_rk3_step, sbli_tgv_init, sbli_num_variants, sbli_variant_info,
                   sbli_set_tuning, sbli_get_tuning, sbli_autotune)

__all__ = ["Solver", "make_params", "SbliError", "sbli_init", "sbli_destroy", "sbli_last_error",
           "sbli_tgv_init", "sbli_rhs", "sbli_rk3_step", "sbli_diagnostics", "sbli_params",
           "sbli_num_variants", "sbli_variant_info", "sbli_set_tuning", "sbli_get_tuning",
           "sbli_autotune"]

DIAG_NAMES = ("Ek", "enstrophy", "rho", "rhou", "rhov", "rhow", "rhoE")


_BC = {"periodic": _lib.SBLI_BC_PERIODIC, "symmetry": _lib.SBLI_BC_SYMMETRY,
       0: _lib.SBLI_BC_PERIODIC, 1: _lib.SBLI_BC_SYMMETRY}


def make_params(n, order=4, dtype="f64", Re=1600.0, Mach=0.1, Pr=0.71, gamma=1.4, length=None,
                bc=("periodic", "periodic", "periodic")):
    """sbli_params for an n = (nx, ny, nz) (or int) box of side 2*pi (default); bc per
    axis "periodic" or "symmetry" (0 / 1)."""
    if isinstance(n, int):
        n = (n, n, n)
    if length is None:
        length = (2 * math.pi,) * 3
    dt = {"f64": SBLI_F64, "f32": SBLI_F32}[dtype]
    p = sbli_params(int(n[0]), int(n[1]), int(n[2]), float(length[0]), float(length[1]),
                    float(length[2]), float(Re), float(Mach), float(Pr), float(gamma), int(order), dt)
    for d in range(3):
        p.bc[d] = _BC[bc[d]]
    return p


class Solver:
    """One box (periodic or with symmetry boundaries per axis) on the current HIP device
    and stream.

    State tensors are torch tensors of shape (5, nz, ny, nx), dtype float64 or
    float32, on the GPU, contiguous.
    """

    def __init__(self, n, order=4, dtype="f64", Re=1600.0, Mach=0.1, Pr=0.71, gamma=1.4,
                 length=None, stream=None, bc=("periodic", "periodic", "periodic")):
        import torch
        self.torch = torch
        self.params = make_params(n, order, dtype, Re, Mach, Pr, gamma, length, bc)
        self.shape = (5, self.params.nz, self.params.ny, self.params.nx)
        self.dtype = torch.float64 if dtype == "f64" else torch.float32
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        self.ctx = sbli_init(self.params, stream.cuda_stream)

    def close(self):
        if self.ctx:
            sbli_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def empty_state(self):
        return self.torch.empty(self.shape, dtype=self.dtype, device="cuda")

    def _check_state(self, t, name):
        if not (t.is_cuda and t.is_contiguous() and tuple(t.shape) == self.shape and t.dtype == self.dtype):
            raise ValueError("%s must be a contiguous CUDA tensor of shape %r and dtype %s"
                             % (name, self.shape, self.dtype))

    def tgv_init(self, q, phase=None):
        self._check_state(q, "q")
        sbli_tgv_init(self.ctx, q, phase)
        return q

    def rhs(self, q, out=None):
        self._check_state(q, "q")
        if out is None:
            out = self.empty_state()
        self._check_state(out, "out")
        sbli_rhs(self.ctx, q, out)
        return out

    def rk3_step(self, q, q_tmp, dq, dt, nsteps=1):
        for t, nm in ((q, "q"), (q_tmp, "q_tmp"), (dq, "dq")):
            self._check_state(t, nm)
        sbli_rk3_step(self.ctx, q, q_tmp, dq, dt, nsteps)
        return q

    def diagnostics(self, q, check=True):
        self._check_state(q, "q")
        vals, code = sbli_diagnostics(self.ctx, q, check=check)
        return dict(zip(DIAG_NAMES, vals)), code

    # ---- launch tuning ----
    def variants(self):
        return [sbli_variant_info(self.ctx, v) for v in range(sbli_num_variants(self.ctx))]

    def set_tuning(self, variant, zchunk):
        sbli_set_tuning(self.ctx, variant, zchunk)

    def get_tuning(self):
        return sbli_get_tuning(self.ctx)

    def autotune(self, reps=2, force=False, path=None):
        kw = {} if path is None else {"path": path}
        return tuning.autotune(self, reps=reps, force=force, **kw)


class Batch:
    """An ensemble of periodic Taylor-Green boxes on the current HIP device and stream.

    `instances` is a list of dicts with keys n, Re, Mach, Pr, gamma, dt, phase
    (see synth.batch_instances).  States are flat torch tensors holding every box
    back to back; `view(q, i)` gives box i as a (5, n, n, n) tensor.
    """

    def __init__(self, instances, order=4, dtype="f32", stream=None):
        import torch
        self.torch = torch
        self.instances = [dict(d) for d in instances]
        self.count = len(instances)
        self.order = order
        self.dtype = torch.float64 if dtype == "f64" else torch.float32
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        recs = [_lib.sbli_instance(int(d["n"]), float(d["Re"]), float(d["Mach"]), float(d["Pr"]),
                                   float(d["gamma"]), float(d["dt"]),
                                   (ctypes_double3(d.get("phase", (0.0, 0.0, 0.0)))))
                for d in instances]
        self.b = _lib.sbli_batch_init(recs, order, SBLI_F64 if dtype == "f64" else SBLI_F32,
                                      stream.cuda_stream)
        self.offsets = _lib.sbli_batch_layout(self.b, self.count)
        self.total = self.offsets[-1]

    def close(self):
        if self.b:
            _lib.sbli_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def points(self):
        return sum(int(d["n"]) ** 3 for d in self.instances)

    def empty_state(self):
        return self.torch.empty(self.total, dtype=self.dtype, device="cuda")

    def view(self, q, i):
        n = int(self.instances[i]["n"])
        return q[self.offsets[i]:self.offsets[i + 1]].view(5, n, n, n)

    def _chk(self, *ts):
        for t in ts:
            if not (t.is_cuda and t.is_contiguous() and t.numel() == self.total and t.dtype == self.dtype):
                raise ValueError("batch states must be contiguous CUDA tensors of %d elements, dtype %s"
                                 % (self.total, self.dtype))

    def tgv_init(self, q):
        self._chk(q)
        _lib.sbli_batch_tgv_init(self.b, q)
        return q

    def step(self, q, q_tmp, dq, nsteps=1):
        self._chk(q, q_tmp, dq)
        _lib.sbli_batch_step(self.b, q, q_tmp, dq, nsteps)
        return q

    def step_sequential(self, q, q_tmp, dq, nsteps=1):
        self._chk(q, q_tmp, dq)
        _lib.sbli_batch_step_sequential(self.b, q, q_tmp, dq, nsteps)
        return q

    def capture(self, q, q_tmp, dq, nsteps):
        self._chk(q, q_tmp, dq)
        _lib.sbli_batch_capture(self.b, q, q_tmp, dq, nsteps)

    def launch(self):
        _lib.sbli_batch_launch(self.b)

    def diagnostics(self, q, check=True):
        self._chk(q)
        return _lib.sbli_batch_diagnostics(self.b, q, self.count, check=check)

    def set_tuning(self, variant, zmax):
        _lib.sbli_batch_set_tuning(self.b, variant, zmax)

    def get_tuning(self):
        return _lib.sbli_batch_get_tuning(self.b)

    def autotune(self, reps=2):
        q, qt, dq = self.empty_state(), self.empty_state(), self.empty_state()
        self.tgv_init(q)
        ms = _lib.sbli_batch_autotune(self.b, q, qt, dq, reps)
        del q, qt, dq
        return ms


def ctypes_double3(v):
    import ctypes
    return (ctypes.c_double * 3)(*[float(x) for x in v])
