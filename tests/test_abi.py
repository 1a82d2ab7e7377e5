"""Host-side checks of the C ABI (no GPU needed): every function declared in
include/*.h is exported by libsbli.so, and argument validation fails cleanly."""
import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = []
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names += re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*(sbli_[a-z0-9_]+)\s*\(", text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    from paper_1609_01277_amd import _lib, build as libbuild
    if not libbuild.is_current():
        import __graft_entry__
        __graft_entry__.build()
    return _lib.load()


def test_header_declares_the_core_calls():
    names = declared_functions()
    for core in ("sbli_init", "sbli_rhs", "sbli_rk3_step", "sbli_diagnostics", "sbli_tgv_init",
                 "sbli_destroy", "sbli_last_error"):
        assert core in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.parametrize("kw,msg", [
    (dict(order=5), "order"),
    (dict(order=3), "order"),
    (dict(n=8, order=4), ">= 9"),
    (dict(n=16, order=8), ">= 17"),
    (dict(Re=0.0), "Re"),
    (dict(Mach=-1.0), "Re, Mach"),
    (dict(gamma=1.0), "gamma"),
    (dict(Pr=float("nan")), "Pr"),
])
def test_init_rejects_bad_params(lib, kw, msg):
    import paper_1609_01277_amd as sbli
    n = kw.pop("n", 32)
    p = sbli.make_params(n, **kw)
    with pytest.raises(sbli.SbliError) as ei:
        sbli.sbli_init(p)
    assert ei.value.code == sbli.SBLI_ERR_ARG
    assert msg in str(ei.value)


def test_init_rejects_bad_boundary_condition(lib):
    import paper_1609_01277_amd as sbli
    p = sbli.make_params(32, bc=("symmetry", "periodic", "symmetry"))
    assert list(p.bc) == [1, 0, 1]
    p.bc[2] = 5
    with pytest.raises(sbli.SbliError) as ei:
        sbli.sbli_init(p)
    assert ei.value.code == sbli.SBLI_ERR_ARG and "bc[2]" in str(ei.value)


def test_init_rejects_bad_dtype_and_null(lib):
    import paper_1609_01277_amd as sbli
    p = sbli.make_params(32)
    p.dtype = 7
    with pytest.raises(sbli.SbliError) as ei:
        sbli.sbli_init(p)
    assert ei.value.code == sbli.SBLI_ERR_ARG
    out = ctypes.c_void_p()
    assert lib.sbli_init(None, None, ctypes.byref(out)) == sbli.SBLI_ERR_ARG
    assert out.value is None
    # NULL-context calls fail with an argument error, not a crash
    assert lib.sbli_rhs(None, None, None) == sbli.SBLI_ERR_ARG
    assert lib.sbli_rk3_step(None, None, None, None, 0.1, 1) == sbli.SBLI_ERR_ARG
    assert lib.sbli_destroy(None) == sbli.SBLI_OK


def test_closure_kernel_exports_validate_arguments(lib):
    """Shape queries and the argument checks of the per-kernel closure calls.  Every call
    below fails (or returns) on the host before any device work; the non-NULL pointers
    are never dereferenced."""
    from paper_1609_01277_amd import closure
    import paper_1609_01277_amd as sbli
    L = closure._L()
    ERR = sbli.SBLI_ERR_ARG
    assert [L.sbli_conv3d_cpad(c) for c in (1, 5, 8, 9, 32)] == [8, 8, 8, 32, 32]
    assert L.sbli_conv3d_cpad(0) == ERR and L.sbli_conv3d_cpad(33) == ERR
    assert L.sbli_conv3d_packed_width(5) == 224 and L.sbli_conv3d_packed_width(32) == 864
    assert L.sbli_conv3d_bwd_weight_work_bytes(32) == 4 * (512 * 32 * 864 + 512 * 32)
    assert L.sbli_conv3d_bwd_weight_work_bytes(5) == 4 * (512 * 32 * 224 + 512 * 32)
    assert L.sbli_conv3d_bwd_weight_work_bytes(40) == ERR
    assert L.sbli_mse_grad_work_bytes(64, 4) == 8 * (4 * 64 ** 3 // 256)
    assert L.sbli_mse_grad_work_bytes(48, 1) == ERR
    assert L.sbli_net_stream(None) is None

    d = ctypes.c_void_p(0x10000)       # stands for a device pointer; never touched

    def msg():
        return L.sbli_net_last_error(None).decode()

    assert L.sbli_conv3d_fwd(None, 5, d, d, 32, 64, 1, 1, d, d, None) == ERR
    assert L.sbli_conv3d_fwd(d, 5, d, d, 32, 48, 1, 1, d, d, None) == ERR and "multiple of 32" in msg()
    assert L.sbli_conv3d_fwd(d, 5, d, d, 5, 64, 1, closure.ACT_GELU, d, d, None) == ERR and "cout = 32" in msg()
    assert L.sbli_conv3d_fwd(d, 5, d, d, 32, 64, 1, 7, d, d, None) == ERR and "act" in msg()
    assert L.sbli_conv3d_fwd(d, 40, d, d, 32, 64, 1, 1, d, d, None) == ERR
    assert L.sbli_conv3d_fwd(d, 5, d, d, 32, 64, 0, 1, d, d, None) == ERR and "batch" in msg()
    assert L.sbli_conv3d_pack(d, 5, 32, None, None, None) == ERR
    assert L.sbli_conv3d_bwd_data(d, 0, d, 64, 1, None, d, None) == ERR
    assert L.sbli_conv3d_bwd_weight(d, 32, d, 32, 64, 1, d, None, d, 1024, None) == ERR and "work" in msg()
    assert L.sbli_mse_grad(d, 5, d, d, 64, 1, d, d, d, 1 << 20, None) == ERR and "ystride" in msg()
    assert L.sbli_mse_grad(d, 8, d, d, 64, 4, d, d, d, 8, None) == ERR and "work" in msg()
    assert L.sbli_adam_step(d, d, d, d, 10, 1e-3, 0, None) == ERR
    assert L.sbli_adam_step(d, d, d, d, 10, 0.0, 1, None) == ERR
    assert L.sbli_adam_step(d, d, d, d, 0, 1e-3, 1, None) == sbli.SBLI_OK
    assert L.sbli_gelu_bwd(d, d, -1, d, None) == ERR
    assert L.sbli_gelu_bwd(d, d, 0, d, None) == sbli.SBLI_OK
    assert L.sbli_net_set_conservative(None, 1) == ERR and "NULL" in msg()
