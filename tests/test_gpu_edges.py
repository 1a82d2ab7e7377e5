"""Degenerate cases of the stencil path on the GPU, against the oracle.

- The smallest grid each order accepts (2 * order + 1 points per axis, so the
  widest stencil reaches every point of the axis and wraps), periodic and with
  symmetry boundaries, through every launch variant and with a z-chunk of one
  plane as well as the whole axis: residual and two RK3 steps within 1e-12 of
  the oracle per field.
- nsteps = 0: the state is left bitwise unchanged.
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


CASES = [(order, (0, 0, 0)) for order in (2, 4, 6, 8, 10, 12)] + [(4, (1, 0, 1)), (8, (0, 1, 1))]


@pytest.mark.parametrize("order,bc", CASES)
def test_smallest_grid_every_variant_matches_oracle(order, bc):
    sbli, torch = _sbli()
    m = 2 * order + 1
    n = (m, m + 1, m)                # the minimum on x and z, one more on y
    length = tuple(math.pi if s else 2 * math.pi for s in bc)
    q0 = synth.random_conservative_state(n, seed=40 + order, mom=0.4)
    p = oracle.Params(n=n, length=length, order=order, Re=80.0, Mach=0.3, bc=bc)
    Rref = oracle.rhs(q0, p)
    dt = 1e-3
    qref = oracle.rk3(q0, p, dt, 2)
    s = sbli.Solver(n, order=order, Re=80.0, Mach=0.3, length=length, bc=bc)
    qd0 = torch.from_numpy(q0).cuda()
    qt, dq = s.empty_state(), s.empty_state()
    for v in range(len(s.variants())):
        for zc in (1, n[2]):
            s.set_tuning(v, zc)
            R = s.rhs(qd0).cpu().numpy()
            errs = rel_err(R, Rref)
            assert max(errs) <= TOL64, (v, zc, errs)
            q = qd0.clone()
            s.rk3_step(q, qt, dq, dt, 2)
            errs = rel_err(q.cpu().numpy(), qref)
            assert max(errs) <= TOL64, (v, zc, errs)
    s.close()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_zero_steps_leave_the_state_unchanged(dtype):
    sbli, torch = _sbli()
    n = (20, 18, 22)
    s = sbli.Solver(n, order=4, dtype=dtype, **synth.TGV)
    q = s.tgv_init(s.empty_state())
    before = q.clone()
    s.rk3_step(q, s.empty_state(), s.empty_state(), 1e-3, 0)
    torch.cuda.synchronize()
    assert torch.equal(q, before)
    s.close()
