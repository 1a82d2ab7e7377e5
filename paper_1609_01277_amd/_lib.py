"""ctypes binding of libsbli.so: argument marshalling only.

Every function here has the name of the C entry point it wraps (include/sbli.h)
and does nothing but convert arguments: all arithmetic of the solver runs in the
HIP kernels of libsbli.so.  The library must have been built (build.py); there is
no fallback of any kind when it is missing.
"""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsbli.so")

SBLI_OK = 0
SBLI_ERR_ARG = -1
SBLI_ERR_HIP = -2
SBLI_ERR_NONFINITE = -3
SBLI_ERR_ALLOC = -4
SBLI_ERR_UNSUPPORTED = -5
SBLI_F64 = 0
SBLI_F32 = 1


class SbliError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("sbli error %d: %s" % (code, msg))
        self.code = code


class sbli_params(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
                ("lx", ctypes.c_double), ("ly", ctypes.c_double), ("lz", ctypes.c_double),
                ("Re", ctypes.c_double), ("Mach", ctypes.c_double), ("Pr", ctypes.c_double),
                ("gamma", ctypes.c_double), ("order", ctypes.c_int), ("dtype", ctypes.c_int),
                ("bc", ctypes.c_int * 3)]

SBLI_BC_PERIODIC = 0
SBLI_BC_SYMMETRY = 1


_lib = None


def load():
    """Load libsbli.so (raises ImportError if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libsbli.so is not built (%s); run __graft_entry__.build() or "
                          "python paper_1609_01277_amd/build.py" % LIB_PATH)
    from . import build as _build
    if not _build.is_current():
        raise ImportError("libsbli.so (%s) was not built from the current sources under csrc/ and "
                          "include/; rebuild it with __graft_entry__.build() or "
                          "python paper_1609_01277_amd/build.py" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    vp = ctypes.c_void_p
    lib.sbli_init.argtypes = [ctypes.POINTER(sbli_params), vp, ctypes.POINTER(vp)]
    lib.sbli_destroy.argtypes = [vp]
    lib.sbli_last_error.argtypes = [vp]
    lib.sbli_last_error.restype = ctypes.c_char_p
    lib.sbli_tgv_init.argtypes = [vp, vp, ctypes.POINTER(ctypes.c_double)]
    lib.sbli_rhs.argtypes = [vp, vp, vp]
    lib.sbli_rk3_step.argtypes = [vp, vp, vp, vp, ctypes.c_double, ctypes.c_int]
    lib.sbli_diagnostics.argtypes = [vp, vp, ctypes.POINTER(ctypes.c_double)]
    ip = ctypes.POINTER(ctypes.c_int)
    lib.sbli_num_variants.argtypes = [vp]
    lib.sbli_variant_info.argtypes = [vp, ctypes.c_int, ip]
    lib.sbli_set_tuning.argtypes = [vp, ctypes.c_int, ctypes.c_int]
    lib.sbli_get_tuning.argtypes = [vp, ip, ip]
    lib.sbli_autotune.argtypes = [vp, vp, vp, vp, ctypes.c_double, ctypes.c_int,
                                  ctypes.POINTER(ctypes.c_double)]
    for name in ("sbli_init", "sbli_destroy", "sbli_tgv_init", "sbli_rhs", "sbli_rk3_step",
                 "sbli_diagnostics", "sbli_num_variants", "sbli_variant_info", "sbli_set_tuning",
                 "sbli_get_tuning", "sbli_autotune"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _check(code, ctx):
    if code != SBLI_OK:
        msg = load().sbli_last_error(ctx)
        raise SbliError(code, msg.decode() if msg else "")
    return code


def _ptr(x):
    """Device address of a torch tensor, or an int address, or None."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


def sbli_init(params, stream=None):
    """Create a context; returns its handle (int).  `stream` is a HIP stream handle (int) or None."""
    ctx = ctypes.c_void_p()
    code = load().sbli_init(ctypes.byref(params), stream, ctypes.byref(ctx))
    _check(code, None)
    return ctx.value


def sbli_destroy(ctx):
    return _check(load().sbli_destroy(ctx), None)


def sbli_last_error(ctx):
    msg = load().sbli_last_error(ctx)
    return msg.decode() if msg else ""


def sbli_tgv_init(ctx, q, phase=None):
    ph = None if phase is None else (ctypes.c_double * 3)(*[float(v) for v in phase])
    return _check(load().sbli_tgv_init(ctx, _ptr(q), ph), ctx)


def sbli_rhs(ctx, q, rhs):
    return _check(load().sbli_rhs(ctx, _ptr(q), _ptr(rhs)), ctx)


def sbli_rk3_step(ctx, q, q_tmp, dq, dt, nsteps):
    return _check(load().sbli_rk3_step(ctx, _ptr(q), _ptr(q_tmp), _ptr(dq), float(dt), int(nsteps)), ctx)


def sbli_diagnostics(ctx, q, check=True):
    """Returns (list of 7 doubles, status code).  Raises on errors other than NONFINITE
    unless check is False."""
    out = (ctypes.c_double * 7)()
    code = load().sbli_diagnostics(ctx, _ptr(q), out)
    if code not in (SBLI_OK, SBLI_ERR_NONFINITE) or (check and code != SBLI_OK):
        _check(code, ctx)
    return list(out), code


def sbli_num_variants(ctx):
    n = load().sbli_num_variants(ctx)
    if n < 0:
        _check(n, ctx)
    return n


def sbli_variant_info(ctx, variant):
    info = (ctypes.c_int * 7)()
    _check(load().sbli_variant_info(ctx, int(variant), info), ctx)
    return tuple(info)


def sbli_set_tuning(ctx, variant, zchunk):
    return _check(load().sbli_set_tuning(ctx, int(variant), int(zchunk)), ctx)


def sbli_get_tuning(ctx):
    v, z = ctypes.c_int(), ctypes.c_int()
    _check(load().sbli_get_tuning(ctx, ctypes.byref(v), ctypes.byref(z)), ctx)
    return v.value, z.value


def sbli_autotune(ctx, q, q_tmp, dq, dt, reps=2):
    ms = ctypes.c_double()
    _check(load().sbli_autotune(ctx, _ptr(q), _ptr(q_tmp), _ptr(dq), float(dt), int(reps),
                                ctypes.byref(ms)), ctx)
    return ms.value


class sbli_instance(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("Re", ctypes.c_double), ("Mach", ctypes.c_double),
                ("Pr", ctypes.c_double), ("gamma", ctypes.c_double), ("dt", ctypes.c_double),
                ("phase", ctypes.c_double * 3)]


_batch_ready = False


def _batch_lib():
    global _batch_ready
    lib = load()
    if not _batch_ready:
        vp = ctypes.c_void_p
        ip = ctypes.POINTER(ctypes.c_int)
        lib.sbli_batch_init.argtypes = [ctypes.POINTER(sbli_instance), ctypes.c_int, ctypes.c_int,
                                        ctypes.c_int, vp, ctypes.POINTER(vp)]
        lib.sbli_batch_destroy.argtypes = [vp]
        lib.sbli_batch_last_error.argtypes = [vp]
        lib.sbli_batch_last_error.restype = ctypes.c_char_p
        lib.sbli_batch_layout.argtypes = [vp, ctypes.POINTER(ctypes.c_size_t)]
        lib.sbli_batch_tgv_init.argtypes = [vp, vp]
        for name in ("sbli_batch_step", "sbli_batch_step_sequential", "sbli_batch_capture"):
            getattr(lib, name).argtypes = [vp, vp, vp, vp, ctypes.c_int]
        lib.sbli_batch_launch.argtypes = [vp]
        lib.sbli_batch_diagnostics.argtypes = [vp, vp, ctypes.POINTER(ctypes.c_double)]
        lib.sbli_batch_set_tuning.argtypes = [vp, ctypes.c_int, ctypes.c_int]
        lib.sbli_batch_get_tuning.argtypes = [vp, ip, ip]
        lib.sbli_batch_autotune.argtypes = [vp, vp, vp, vp, ctypes.c_int, ctypes.POINTER(ctypes.c_double)]
        for name in ("sbli_batch_init", "sbli_batch_destroy", "sbli_batch_layout", "sbli_batch_tgv_init",
                     "sbli_batch_step", "sbli_batch_step_sequential", "sbli_batch_capture",
                     "sbli_batch_launch", "sbli_batch_diagnostics", "sbli_batch_set_tuning",
                     "sbli_batch_get_tuning", "sbli_batch_autotune"):
            getattr(lib, name).restype = ctypes.c_int
        _batch_ready = True
    return lib


def _bcheck(code, b):
    if code not in (SBLI_OK,):
        msg = _batch_lib().sbli_batch_last_error(b)
        raise SbliError(code, msg.decode() if msg else "")
    return code


def sbli_batch_init(instances, order, dtype, stream=None):
    arr = (sbli_instance * len(instances))(*instances)
    out = ctypes.c_void_p()
    _bcheck(_batch_lib().sbli_batch_init(arr, len(instances), int(order), int(dtype), stream,
                                         ctypes.byref(out)), None)
    return out.value


def sbli_batch_destroy(b):
    return _bcheck(_batch_lib().sbli_batch_destroy(b), None)


def sbli_batch_layout(b, count):
    off = (ctypes.c_size_t * (count + 1))()
    _bcheck(_batch_lib().sbli_batch_layout(b, off), b)
    return list(off)


def sbli_batch_tgv_init(b, q):
    return _bcheck(_batch_lib().sbli_batch_tgv_init(b, _ptr(q)), b)


def sbli_batch_step(b, q, q_tmp, dq, nsteps):
    return _bcheck(_batch_lib().sbli_batch_step(b, _ptr(q), _ptr(q_tmp), _ptr(dq), int(nsteps)), b)


def sbli_batch_step_sequential(b, q, q_tmp, dq, nsteps):
    return _bcheck(_batch_lib().sbli_batch_step_sequential(b, _ptr(q), _ptr(q_tmp), _ptr(dq), int(nsteps)), b)


def sbli_batch_capture(b, q, q_tmp, dq, nsteps):
    return _bcheck(_batch_lib().sbli_batch_capture(b, _ptr(q), _ptr(q_tmp), _ptr(dq), int(nsteps)), b)


def sbli_batch_launch(b):
    return _bcheck(_batch_lib().sbli_batch_launch(b), b)


def sbli_batch_diagnostics(b, q, count, check=True):
    out = (ctypes.c_double * (7 * count))()
    code = _batch_lib().sbli_batch_diagnostics(b, _ptr(q), out)
    if code not in (SBLI_OK, SBLI_ERR_NONFINITE) or (check and code != SBLI_OK):
        _bcheck(code, b)
    return [list(out[7 * i:7 * i + 7]) for i in range(count)], code


def sbli_batch_set_tuning(b, variant, zmax):
    return _bcheck(_batch_lib().sbli_batch_set_tuning(b, int(variant), int(zmax)), b)


def sbli_batch_get_tuning(b):
    v, z = ctypes.c_int(), ctypes.c_int()
    _bcheck(_batch_lib().sbli_batch_get_tuning(b, ctypes.byref(v), ctypes.byref(z)), b)
    return v.value, z.value


def sbli_batch_autotune(b, q, q_tmp, dq, reps=2):
    ms = ctypes.c_double()
    _bcheck(_batch_lib().sbli_batch_autotune(b, _ptr(q), _ptr(q_tmp), _ptr(dq), int(reps),
                                             ctypes.byref(ms)), b)
    return ms.value
