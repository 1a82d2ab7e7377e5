"""Orders 10 and 12 of the Navier-Stokes path (paper Sec. "Discretisation schemes":
central differences of arbitrary even order), and the staged form of the stage kernel
that serves them.

- Orders 10 and 12 against the FP64 oracle: residual of a random state, RK3 steps of
  the Taylor-Green state, diagnostics, and a box with symmetry boundaries; 1e-12
  relative per field (momentum normalised by its largest component).
- The staged form is also a launch variant of orders 2..8, where it computes the same
  arithmetic per point as the fused stage kernel: every variant agrees bit for bit
  (`test_gpu_variants.py` covers periodic boxes; here a box with symmetry boundaries
  and FP32).
"""
import math

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

TOL64 = 1e-12


def _sbli():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a HIP device")
    import paper_1609_01277_amd as sbli
    return sbli, torch


def rel_err(got, ref):
    mom = np.abs(ref[1:4]).max()
    return [np.abs(got[f] - ref[f]).max() / max(mom if f in (1, 2, 3) else np.abs(ref[f]).max(), 1e-300)
            for f in range(5)]


# (70, 40, 26) spans 5 x 3 of the 16 x 16 tiles of both steps, so tile pairs cross tile
# rows and the ragged last tiles hold mirrored or wrapped columns.  With nz = 100 the
# z-marching nested-field step runs 64 planes and then 36 (a run starting inside the
# box, and a short last run).
@pytest.mark.parametrize("order,n", [(10, (26, 27, 29)), (12, (26, 27, 29)), (12, (70, 40, 26)),
                                     (10, (26, 27, 100)), (12, (26, 27, 100))])
def test_high_order_rhs_matches_oracle(order, n):
    sbli, torch = _sbli()
    q0 = synth.random_conservative_state(n, seed=40 + order, mom=0.3)
    s = sbli.Solver(n, order=order, **synth.TGV)
    assert s.variants() == [(0, 0, 0, 0, 0, 0, 0)]      # the staged form only
    R = s.rhs(torch.from_numpy(q0).cuda()).cpu().numpy()
    errs = rel_err(R, oracle.rhs(q0, oracle.Params(n=n, order=order, **synth.TGV)))
    assert max(errs) <= TOL64, errs


@pytest.mark.parametrize("order", [10, 12])
def test_high_order_rk3_and_diagnostics_match_oracle(order):
    sbli, torch = _sbli()
    n = 28
    p = oracle.Params(n=(n, n, n), order=order, **synth.TGV)
    s = sbli.Solver(n, order=order, **synth.TGV)
    qo = oracle.tgv_init(p)
    q = torch.from_numpy(qo.copy()).cuda()
    dt = 3.385e-3 * 32 / n        # the 32^3 Taylor-Green step at the same Courant number
    for step in range(3):
        s.rk3_step(q, s.empty_state(), s.empty_state(), dt, 1)
        qo = oracle.rk3(qo, p, dt, 1)
        errs = rel_err(q.cpu().numpy(), qo)
        assert max(errs) <= TOL64, (step, errs)
    d, code = s.diagnostics(q, check=False)
    assert code == 0
    do, _ = oracle.diagnostics(q.cpu().numpy(), p)
    got = np.array([d[k] for k in ("Ek", "enstrophy", "rho", "rhou", "rhov", "rhow", "rhoE")])
    assert np.abs(got[:2] - do[:2]).max() <= 1e-12 * np.abs(do[:2]).max()
    assert np.abs(got[2:] - do[2:]).max() <= 1e-12 * np.abs(do[2:]).max()


def test_order10_symmetry_matches_oracle():
    sbli, torch = _sbli()
    n, bc = (30, 26, 28), (1, 0, 1)
    length = tuple(math.pi if b else 2 * math.pi for b in bc)
    q0 = synth.random_conservative_state(n, seed=77, mom=0.4)
    p = oracle.Params(n=n, length=length, order=10, Re=80.0, Mach=0.3, bc=bc)
    s = sbli.Solver(n, order=10, Re=80.0, Mach=0.3, length=length, bc=bc)
    R = s.rhs(torch.from_numpy(q0).cuda()).cpu().numpy()
    assert max(rel_err(R, oracle.rhs(q0, p))) <= TOL64
    q = torch.from_numpy(q0).cuda()
    s.rk3_step(q, s.empty_state(), s.empty_state(), 1e-3, 2)
    errs = rel_err(q.cpu().numpy(), oracle.rk3(q0, p, 1e-3, 2))
    assert max(errs) <= TOL64, errs


# (36, 20, 34) has 3 x 2 tiles of 16 x 16 columns, so tile pairs of the staged
# launches span two tile rows; (36, 40, 22) has 3 x 3, which leaves one tile unpaired.
@pytest.mark.parametrize("dtype,bc,order,n", [("f64", (1, 1, 0), 4, (36, 20, 34)), ("f64", (0, 1, 1), 8, (36, 20, 34)),
                                              ("f32", (1, 0, 1), 4, (36, 20, 34)), ("f64", (0, 0, 0), 6, (36, 40, 22)),
                                              ("f64", (1, 0, 1), 8, (36, 40, 22))])
def test_staged_form_bitwise_equals_fused(dtype, bc, order, n):
    sbli, torch = _sbli()
    length = tuple(math.pi if b else 2 * math.pi for b in bc)
    q0 = synth.random_conservative_state(n, seed=9 + order, mom=0.4)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    s = sbli.Solver(n, order=order, dtype=dtype, Re=80.0, Mach=0.3, length=length, bc=bc)
    variants = s.variants()
    staged = len(variants) - 1
    assert variants[staged] == (0, 0, 0, 0, 0, 0, 0)
    out = {}
    for v in (0, staged):
        s.set_tuning(v, n[2])
        q = torch.from_numpy(q0).to(tdt).cuda()
        R = s.rhs(q).cpu().numpy()
        s.rk3_step(q, s.empty_state(), s.empty_state(), 1e-3, 2)
        out[v] = (R, q.cpu().numpy())
    assert np.array_equal(out[0][0], out[staged][0])
    assert np.array_equal(out[0][1], out[staged][1])


def test_high_order_limits():
    sbli, torch = _sbli()
    with pytest.raises(Exception):
        sbli.Solver(40, order=14, **synth.TGV)
    with pytest.raises(Exception):
        sbli.Solver(24, order=12, **synth.TGV)      # needs n >= 2 * order + 1 = 25
    with pytest.raises(Exception):
        sbli.Batch([dict(n=32, Re=1600.0, Mach=0.1, Pr=0.71, gamma=1.4, dt=1e-3)], order=10)
