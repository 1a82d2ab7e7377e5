"""ctypes binding of the scalar advection-diffusion entry points (include/sbli_scalar.h).

Argument marshalling only.  Arrays are FP64 torch tensors on the GPU, shaped
(n[2], n[1], n[0]) or flat.
"""
import ctypes

from . import _lib

_ready = False


class sbli_scalar_params(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int * 3), ("length", ctypes.c_double * 3), ("order", ctypes.c_int),
                ("c", ctypes.c_double * 3), ("k", ctypes.c_double)]


def _L():
    global _ready
    lib = _lib.load()
    if not _ready:
        vp = ctypes.c_void_p
        pp = ctypes.POINTER(sbli_scalar_params)
        lib.sbli_scalar_rhs.argtypes = [pp, vp, vp, vp, vp]
        lib.sbli_scalar_rk3.argtypes = [pp, vp, vp, vp, vp, ctypes.c_double, ctypes.c_int, vp]
        lib.sbli_scalar_last_error.argtypes = []
        lib.sbli_scalar_last_error.restype = ctypes.c_char_p
        lib.sbli_scalar_rhs.restype = ctypes.c_int
        lib.sbli_scalar_rk3.restype = ctypes.c_int
        _ready = True
    return lib


def params(n, length, order, c=(0.0, 0.0, 0.0), k=0.0):
    n = list(n) + [1] * (3 - len(n))
    length = list(length) + [1.0] * (3 - len(length))
    c = list(c) + [0.0] * (3 - len(c))
    return sbli_scalar_params((ctypes.c_int * 3)(*n), (ctypes.c_double * 3)(*length), int(order),
                              (ctypes.c_double * 3)(*c), float(k))


def _check(code):
    if code != _lib.SBLI_OK:
        raise _lib.SbliError(code, _L().sbli_scalar_last_error().decode())


def _ptr(t):
    return None if t is None else t.data_ptr()


def sbli_scalar_rhs(p, phi, source, rhs, stream=None):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream().cuda_stream
    _check(_L().sbli_scalar_rhs(ctypes.byref(p), _ptr(phi), _ptr(source), _ptr(rhs), stream))
    return rhs


def sbli_scalar_rk3(p, phi, phi_tmp, dphi, source, dt, nsteps, stream=None):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream().cuda_stream
    _check(_L().sbli_scalar_rk3(ctypes.byref(p), _ptr(phi), _ptr(phi_tmp), _ptr(dphi), _ptr(source),
                                float(dt), int(nsteps), stream))
    return phi
