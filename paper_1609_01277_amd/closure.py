"""ctypes binding of the learned-closure part of libsbli.so (include/sbli_closure.h).

Argument marshalling only; the network, its training and the box filter run in
the library's HIP kernels.  Device arrays are torch tensors (FP32 planar
[batch][5][n][n][n]); parameters are a flat FP32 vector of 36357 values.
"""
import ctypes

import numpy as np

from . import _lib

N_STATS = 35
_ready = False


def _L():
    global _ready
    lib = _lib.load()
    if not _ready:
        vp = ctypes.c_void_p
        fp = ctypes.POINTER(ctypes.c_float)
        lib.sbli_net_create.argtypes = [ctypes.c_int, ctypes.c_int, vp, ctypes.POINTER(vp)]
        lib.sbli_net_destroy.argtypes = [vp]
        lib.sbli_net_last_error.argtypes = [vp]
        lib.sbli_net_last_error.restype = ctypes.c_char_p
        lib.sbli_net_num_params.argtypes = [vp]
        lib.sbli_net_n.argtypes = [vp]
        lib.sbli_net_set_params.argtypes = [vp, fp]
        lib.sbli_net_get_params.argtypes = [vp, fp]
        lib.sbli_net_get_grads.argtypes = [vp, fp]
        lib.sbli_net_set_stats.argtypes = [vp, fp]
        lib.sbli_net_get_stats.argtypes = [vp, fp]
        lib.sbli_net_channel_stats.argtypes = [vp, vp, ctypes.c_int, ctypes.c_int]
        lib.sbli_net_forward.argtypes = [vp, vp, ctypes.c_int, vp]
        lib.sbli_net_set_conservative.argtypes = [vp, ctypes.c_int]
        lib.sbli_net_gradients.argtypes = [vp, vp, vp, ctypes.c_int, ctypes.POINTER(ctypes.c_double)]
        lib.sbli_net_train_step.argtypes = [vp, vp, vp, ctypes.c_int, ctypes.c_float,
                                            ctypes.POINTER(ctypes.c_double)]
        lib.sbli_net_guard.argtypes = [vp, vp, vp, vp]
        lib.sbli_box_filter.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, vp,
                                        ctypes.c_int, vp]
        lib.sbli_net_stream.argtypes = [vp]
        lib.sbli_net_stream.restype = vp
        ll, i = ctypes.c_longlong, ctypes.c_int
        lib.sbli_conv3d_cpad.argtypes = [i]
        lib.sbli_conv3d_packed_width.argtypes = [i]
        lib.sbli_conv3d_pack.argtypes = [vp, i, i, vp, vp, vp]
        lib.sbli_conv3d_fwd.argtypes = [vp, i, vp, vp, i, i, i, i, vp, vp, vp]
        lib.sbli_conv3d_bwd_data.argtypes = [vp, i, vp, i, i, vp, vp, vp]
        lib.sbli_gelu_bwd.argtypes = [vp, vp, ll, vp, vp]
        lib.sbli_conv3d_bwd_weight_work_bytes.argtypes = [i]
        lib.sbli_conv3d_bwd_weight_work_bytes.restype = ll
        lib.sbli_conv3d_bwd_weight.argtypes = [vp, i, vp, i, i, i, vp, vp, vp, ll, vp]
        lib.sbli_mse_grad_work_bytes.argtypes = [i, i]
        lib.sbli_mse_grad_work_bytes.restype = ll
        lib.sbli_mse_grad.argtypes = [vp, i, vp, vp, i, i, vp, vp, vp, ll, vp]
        lib.sbli_mse_grad_noalloc.argtypes = [vp, i, vp, vp, i, i, vp, vp, vp]
        lib.sbli_mse_grad_noalloc.restype = ctypes.c_int
        lib.sbli_adam_step.argtypes = [vp, vp, vp, vp, i, ctypes.c_float, i, vp]
        for name in ("sbli_conv3d_cpad", "sbli_conv3d_packed_width", "sbli_conv3d_pack", "sbli_conv3d_fwd",
                     "sbli_conv3d_bwd_data", "sbli_gelu_bwd", "sbli_conv3d_bwd_weight", "sbli_mse_grad",
                     "sbli_adam_step"):
            getattr(lib, name).restype = ctypes.c_int
        lib.sbli_closure_attach.argtypes = [vp, vp]
        lib.sbli_closure_counts.argtypes = [vp, ctypes.POINTER(ctypes.c_uint)]
        for name in ("sbli_net_create", "sbli_net_destroy", "sbli_net_num_params", "sbli_net_n",
                     "sbli_net_set_params", "sbli_net_get_params", "sbli_net_get_grads", "sbli_net_set_stats",
                     "sbli_net_get_stats", "sbli_net_channel_stats", "sbli_net_forward", "sbli_net_gradients",
                     "sbli_net_train_step", "sbli_net_guard", "sbli_box_filter", "sbli_closure_attach",
                     "sbli_closure_counts"):
            getattr(lib, name).restype = ctypes.c_int
        _ready = True
    return lib


def _check(code, net=None):
    if code != _lib.SBLI_OK:
        msg = _L().sbli_net_last_error(net)
        raise _lib.SbliError(code, msg.decode() if msg else "")


def _fp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


def sbli_box_filter(fine, nf, nfields, ratio, coarse, subtract=False, stream=None):
    """Box-filter planar fields of an nf^3 grid (torch float64/float32) into `coarse` (float32);
    with subtract=True, coarse <- F(fine) - coarse."""
    import torch
    dt = _lib.SBLI_F64 if fine.dtype == torch.float64 else _lib.SBLI_F32
    if stream is None:
        stream = torch.cuda.current_stream().cuda_stream
    _check(_L().sbli_box_filter(fine.data_ptr(), dt, int(nf), int(nfields), int(ratio), coarse.data_ptr(),
                                1 if subtract else 0, stream))
    return coarse


# ---- the network's kernels, one entry point each (device tensors, current stream) ----
ACT_NONE = 0
ACT_GELU = 1


def _stream(stream):
    import torch
    return torch.cuda.current_stream().cuda_stream if stream is None else stream


def _ptr(t):
    return None if t is None else t.data_ptr()


def sbli_conv3d_cpad(channels):
    return _L().sbli_conv3d_cpad(int(channels))


def sbli_conv3d_packed_width(channels):
    return _L().sbli_conv3d_packed_width(int(channels))


def sbli_conv3d_pack(W, cin, cout, Wf, Wb, stream=None):
    _check(_L().sbli_conv3d_pack(W.data_ptr(), int(cin), int(cout), _ptr(Wf), _ptr(Wb), _stream(stream)))


def sbli_conv3d_fwd(x, cin, Wf, b, cout, n, batch, act, pre, h=None, stream=None):
    _check(_L().sbli_conv3d_fwd(x.data_ptr(), int(cin), Wf.data_ptr(), b.data_ptr(), int(cout), int(n), int(batch),
                                int(act), pre.data_ptr(), _ptr(h), _stream(stream)))


def sbli_conv3d_bwd_data(dy, cout, Wb, n, batch, pre, dx, stream=None):
    _check(_L().sbli_conv3d_bwd_data(dy.data_ptr(), int(cout), Wb.data_ptr(), int(n), int(batch), _ptr(pre),
                                     dx.data_ptr(), _stream(stream)))


def sbli_gelu_bwd(g, pre, count, dx, stream=None):
    _check(_L().sbli_gelu_bwd(g.data_ptr(), pre.data_ptr(), int(count), dx.data_ptr(), _stream(stream)))


def sbli_conv3d_bwd_weight_work_bytes(cin):
    return _L().sbli_conv3d_bwd_weight_work_bytes(int(cin))


def sbli_conv3d_bwd_weight(x, cin, dy, cout, n, batch, dW, db, work, stream=None):
    _check(_L().sbli_conv3d_bwd_weight(x.data_ptr(), int(cin), dy.data_ptr(), int(cout), int(n), int(batch),
                                       dW.data_ptr(), _ptr(db), work.data_ptr(),
                                       work.numel() * work.element_size(), _stream(stream)))


def sbli_mse_grad_work_bytes(n, batch):
    return _L().sbli_mse_grad_work_bytes(int(n), int(batch))


def sbli_mse_grad(y, ystride, t, mean_std, n, batch, dy, loss, work, stream=None):
    _check(_L().sbli_mse_grad(y.data_ptr(), int(ystride), t.data_ptr(), mean_std.data_ptr(), int(n), int(batch),
                              dy.data_ptr(), loss.data_ptr(), work.data_ptr(), work.numel() * work.element_size(),
                              _stream(stream)))


def sbli_mse_grad_noalloc(y, ystride, t, mean_std, n, batch, dy, loss, stream=None):
    _check(_L().sbli_mse_grad_noalloc(y.data_ptr(), int(ystride), t.data_ptr(), mean_std.data_ptr(), int(n),
                                      int(batch), dy.data_ptr(), loss.data_ptr(), _stream(stream)))


def sbli_adam_step(p, g, m, v, count, lr, t, stream=None):
    _check(_L().sbli_adam_step(p.data_ptr(), g.data_ptr(), m.data_ptr(), v.data_ptr(), int(count), float(lr),
                               int(t), _stream(stream)))


class ClosureNet:
    """The closure network on the current HIP device and stream."""

    def __init__(self, n=64, max_batch=4, stream=None):
        import torch
        self.torch = torch
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        out = ctypes.c_void_p()
        _check(_L().sbli_net_create(int(n), int(max_batch), stream.cuda_stream, ctypes.byref(out)))
        self.net = out.value
        self.n = n
        self.max_batch = max_batch
        self.nparams = _L().sbli_net_num_params(self.net)

    def close(self):
        if self.net:
            _L().sbli_net_destroy(self.net)
            self.net = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, p):
        p = np.ascontiguousarray(p, dtype=np.float32)
        if p.size != self.nparams:
            raise ValueError("expected %d parameters" % self.nparams)
        _check(_L().sbli_net_set_params(self.net, _fp(p)), self.net)

    def get_params(self):
        p = np.empty(self.nparams, dtype=np.float32)
        _check(_L().sbli_net_get_params(self.net, _fp(p)), self.net)
        return p

    def get_grads(self):
        g = np.empty(self.nparams, dtype=np.float32)
        _check(_L().sbli_net_get_grads(self.net, _fp(g)), self.net)
        return g

    def set_stats(self, s):
        s = np.ascontiguousarray(s, dtype=np.float32)
        if s.size != N_STATS:
            raise ValueError("expected %d statistics" % N_STATS)
        _check(_L().sbli_net_set_stats(self.net, _fp(s)), self.net)

    def get_stats(self):
        s = np.empty(N_STATS, dtype=np.float32)
        _check(_L().sbli_net_get_stats(self.net, _fp(s)), self.net)
        return s

    def channel_stats(self, data, which):
        """Per-field mean/std of planar samples `data` [count][5][n^3] into slot 0 (input) or 1 (output)."""
        count = data.shape[0]
        _check(_L().sbli_net_channel_stats(self.net, data.data_ptr(), int(count), int(which)), self.net)

    def forward(self, q, out=None):
        batch = q.shape[0]
        if out is None:
            out = self.torch.empty_like(q)
        _check(_L().sbli_net_forward(self.net, q.data_ptr(), int(batch), out.data_ptr()), self.net)
        return out

    def set_conservative(self, on=True):
        """Remove each output field's box mean in forward (and in the closure term)."""
        _check(_L().sbli_net_set_conservative(self.net, int(bool(on))), self.net)

    def gradients(self, q, target):
        loss = ctypes.c_double()
        _check(_L().sbli_net_gradients(self.net, q.data_ptr(), target.data_ptr(), int(q.shape[0]),
                                       ctypes.byref(loss)), self.net)
        return loss.value

    def train_step(self, q, target, lr):
        loss = ctypes.c_double()
        _check(_L().sbli_net_train_step(self.net, q.data_ptr(), target.data_ptr(), int(q.shape[0]),
                                        float(lr), ctypes.byref(loss)), self.net)
        return loss.value

    def guard(self, c, flag, counters):
        _check(_L().sbli_net_guard(self.net, c.data_ptr(), flag.data_ptr(), counters.data_ptr()), self.net)


def attach(solver, net):
    """Attach `net` (ClosureNet) to an FP32 Solver (None detaches)."""
    code = _L().sbli_closure_attach(solver.ctx, net.net if net is not None else None)
    if code != _lib.SBLI_OK:
        raise _lib.SbliError(code, _lib.sbli_last_error(solver.ctx))


def counts(solver):
    c = (ctypes.c_uint * 2)()
    code = _L().sbli_closure_counts(solver.ctx, c)
    if code != _lib.SBLI_OK:
        raise _lib.SbliError(code, _lib.sbli_last_error(solver.ctx))
    return c[0], c[1]


# ---- parameter layout helpers (flat vector <-> per-layer arrays) ----
CHANNELS = (5, 32, 32, 5)


def split_params(p):
    """Flat vector -> [(W [o][i][3][3][3], b [o])] per layer."""
    out, off = [], 0
    for ci, co in zip(CHANNELS[:-1], CHANNELS[1:]):
        W = p[off:off + co * ci * 27].reshape(co, ci, 3, 3, 3)
        off += co * ci * 27
        b = p[off:off + co]
        off += co
        out.append((W, b))
    return out


def join_params(layers):
    return np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in layers])
