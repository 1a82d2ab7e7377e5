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
    from paper_1609_01277_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
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
