"""Symmetry boundaries on the GPU (paper Sec. "Boundary conditions").

- Against the oracle's own symmetry-boundary implementation (mirror indexing with the
  parity of every differentiated field): residual, RK3 steps and diagnostics, 1e-12
  relative per field in FP64, 1e-5 in FP32.
- A box of N points with symmetry boundaries against the periodic box of 2N points
  holding the state and its mirror image: for one residual evaluation the kernels
  compute the same operations on the same values, so the two agree bitwise on the
  first N points, for every launch variant of the fused stage kernel.  Over RK3 steps
  the periodic box keeps the mirror symmetry only to rounding (a contracted a*b - c*d
  rounds differently from its mirror image -(c*d - a*b)), so the steps agree to 1e-13.
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


def extend(q, bc):
    out = q.copy()
    for axis, sym in enumerate(bc):
        if sym:
            ax = 3 - axis
            mir = np.flip(out, axis=ax).copy()
            mir[1 + axis] *= -1.0
            out = np.concatenate([out, mir], axis=ax)
    return out


CASES = [((1, 1, 1), 4), ((1, 0, 1), 4), ((0, 1, 0), 8), ((1, 1, 1), 8), ((1, 1, 0), 2), ((0, 0, 1), 6)]


@pytest.mark.parametrize("bc,order", CASES)
def test_symmetry_rhs_and_rk3_match_oracle(bc, order):
    sbli, torch = _sbli()
    n = (36, 20, 34)
    length = tuple(math.pi if s else 2 * math.pi for s in bc)
    q0 = synth.random_conservative_state(n, seed=3 + order, mom=0.4)
    p = oracle.Params(n=n, length=length, order=order, Re=80.0, Mach=0.3, bc=bc)
    s = sbli.Solver(n, order=order, Re=80.0, Mach=0.3, length=length, bc=bc)
    R = s.rhs(torch.from_numpy(q0).cuda()).cpu().numpy()
    assert max(rel_err(R, oracle.rhs(q0, p))) <= TOL64
    q = torch.from_numpy(q0).cuda()
    s.rk3_step(q, s.empty_state(), s.empty_state(), 1e-3, 2)
    errs = rel_err(q.cpu().numpy(), oracle.rk3(q0, p, 1e-3, 2))
    assert max(errs) <= TOL64, errs
    d, code = s.diagnostics(q, check=False)
    do, _ = oracle.diagnostics(q.cpu().numpy(), p)
    got = np.array([d[k] for k in ("Ek", "enstrophy", "rho", "rhou", "rhov", "rhow", "rhoE")])
    assert np.abs(got[:2] - do[:2]).max() <= 1e-12 * np.abs(do[:2]).max()
    assert np.abs(got[2:] - do[2:]).max() <= 1e-12 * np.abs(do[2:]).max()


def test_symmetry_fp32_matches_oracle():
    sbli, torch = _sbli()
    n, bc = (32, 24, 20), (1, 1, 1)
    length = (math.pi,) * 3
    q0 = synth.random_conservative_state(n, seed=8, mom=0.3)
    p = oracle.Params(n=n, length=length, order=4, Re=100.0, Mach=0.3, bc=bc)
    s = sbli.Solver(n, order=4, dtype="f32", Re=100.0, Mach=0.3, length=length, bc=bc)
    q = torch.from_numpy(q0.astype(np.float32)).cuda()
    s.rk3_step(q, s.empty_state(), s.empty_state(), 1e-3, 3)
    errs = rel_err(q.cpu().numpy().astype(np.float64), oracle.rk3(q0.astype(np.float32).astype(np.float64), p, 1e-3, 3))
    assert max(errs) <= 1e-5, errs


@pytest.mark.parametrize("bc,order", [((1, 1, 1), 4), ((1, 0, 1), 8), ((0, 1, 0), 4)])
def test_symmetry_box_equals_mirrored_periodic_box_bitwise(bc, order):
    sbli, torch = _sbli()
    n = (24, 20, 26)
    n2 = tuple(k * (2 if s else 1) for k, s in zip(n, bc))
    length = tuple(math.pi if s else 2 * math.pi for s in bc)
    q0 = synth.random_conservative_state(n, seed=17, mom=0.3)
    qe = extend(q0, bc)
    s = sbli.Solver(n, order=order, Re=200.0, Mach=0.2, length=length, bc=bc)
    pbox = sbli.Solver(n2, order=order, Re=200.0, Mach=0.2, length=(2 * math.pi,) * 3)
    nx, ny, nz = n
    Rp = pbox.rhs(torch.from_numpy(qe).cuda()).cpu().numpy()[:, :nz, :ny, :nx]
    for v in range(len(s.variants())):
        s.set_tuning(v, n[2])
        R = s.rhs(torch.from_numpy(q0).cuda()).cpu().numpy()
        assert np.array_equal(R, Rp), ("rhs", v, s.variants()[v])
    q, qp = torch.from_numpy(q0).cuda(), torch.from_numpy(qe).cuda()
    s.set_tuning(0, 7)
    s.rk3_step(q, s.empty_state(), s.empty_state(), 2e-3, 2)
    pbox.rk3_step(qp, pbox.empty_state(), pbox.empty_state(), 2e-3, 2)
    errs = rel_err(q.cpu().numpy(), qp.cpu().numpy()[:, :nz, :ny, :nx])
    assert max(errs) <= 1e-13, errs


