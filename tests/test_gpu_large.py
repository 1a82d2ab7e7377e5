"""Grids whose state has more elements than a 32-bit index reaches.

Every offset the kernels form (field f at f * P + point) is 64-bit.  These cases
put the last field's elements beyond 2^31 (FP64, 776 x 770 x 768, ragged x and y
tiles) and beyond 2^32 (FP32, 1024^3), run one RK3 step through every launch
variant tested, check the variants bitwise against each other, and compare the
result with the oracle at sampled points that include the box's last point
(element index 5P - 1).
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32_STEP = 1e-6   # as for the 512^3 FP32 step: one step of FP32 rounding, measured <= 2.2e-7


def _sbli():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a HIP device")
    import paper_1609_01277_amd as sbli
    return sbli, torch


def _points(nx, ny, nz, seed):
    rng = np.random.default_rng(seed)
    pts = [(nx - 1, ny - 1, nz - 1), (0, 0, 0), (nx - 2, 3, nz - 1), (5, ny - 1, nz // 2), (nx - 1, ny // 2, 1)]
    pts += [(int(rng.integers(0, nx)), int(rng.integers(0, ny)), int(rng.integers(0, nz))) for _ in range(3)]
    return pts


def _at(torch, q, pts):
    idx = torch.tensor([[z, y, x] for (x, y, z) in pts], device="cuda")
    return q[:, idx[:, 0], idx[:, 1], idx[:, 2]].cpu().numpy().T.astype(np.float64)


def _field_scale(q0):
    scale = np.abs(q0).reshape(5, -1).max(axis=1)
    scale[1:4] = scale[1:4].max()
    return scale


def _step_variants(s, torch, qd0, variants, zchunk, dt):
    """One RK3 step from qd0 with each variant; returns the first result and checks the
    others bitwise against it."""
    qt, dq = s.empty_state(), s.empty_state()
    ref = None
    for v in variants:
        s.set_tuning(v, zchunk)
        q = qd0.clone()
        s.rk3_step(q, qt, dq, dt, 1)
        torch.cuda.synchronize()
        print("variant %d %s done" % (v, s.variants()[v]), flush=True)
        if ref is None:
            ref = q
        else:
            assert torch.equal(q, ref), v
            del q
    del qt, dq
    return ref


def test_fp64_beyond_2_31_elements_every_variant(oracle_mod):
    sbli, torch = _sbli()
    nx, ny, nz, order = 776, 770, 768, 4
    P = nx * ny * nz
    assert 5 * P > 2**31
    dt = synth.tgv_dt(nz)
    p = oracle.Params(n=(nx, ny, nz), order=order, **synth.TGV)
    print("oracle Taylor-Green state %dx%dx%d" % (nx, ny, nz), flush=True)
    q0 = oracle.tgv_init(p)
    s = sbli.Solver((nx, ny, nz), order=order, **synth.TGV)
    qd0 = torch.from_numpy(q0).cuda()
    d0, _ = s.diagnostics(qd0)
    nv = len(s.variants())
    q = _step_variants(s, torch, qd0, list(range(nv)), 192, dt)   # the fused variants and the staged form
    pts = _points(nx, ny, nz, 776)
    ref = oracle.rk3_at_points(q0, p, dt, pts)
    err = (np.abs(_at(torch, q, pts) - ref) / _field_scale(q0)).max()
    assert err <= TOL64, err
    d1, code = s.diagnostics(q)
    assert code == sbli.SBLI_OK
    for name in ("rho", "rhou", "rhov", "rhow", "rhoE"):
        assert abs(d1[name] - d0[name]) < 1e-13 * max(1.0, abs(d0[name])), name
    del q, qd0
    s.close()
    torch.cuda.empty_cache()


def test_fp32_beyond_2_32_elements(oracle_mod):
    sbli, torch = _sbli()
    n, order = 1024, 4
    assert 5 * n**3 > 2**32
    dt = synth.tgv_dt(n)
    p = oracle.Params(n=(n, n, n), order=order, **synth.TGV)
    print("oracle Taylor-Green state %d^3" % n, flush=True)
    q32 = oracle.tgv_init(p).astype(np.float32)
    s = sbli.Solver(n, order=order, dtype="f32", **synth.TGV)
    qd0 = torch.from_numpy(q32).cuda()
    q0 = q32.astype(np.float64)
    del q32
    vs = s.variants()
    # the widest fused tile, a 16x16 one and the staged form
    wide = max(range(len(vs) - 1), key=lambda v: vs[v][0] * vs[v][1])
    sq = next(v for v in range(len(vs) - 1) if vs[v][0] == 16 and vs[v][1] == 16)
    q = _step_variants(s, torch, qd0, [wide, sq, len(vs) - 1], 256, dt)
    pts = _points(n, n, n, 1024)
    ref = oracle.rk3_at_points(q0, p, dt, pts)
    err = (np.abs(_at(torch, q, pts) - ref) / _field_scale(q0)).max(axis=0)
    print("FP32 1024^3 one step: relative error per field %s" % err, flush=True)
    assert err.max() <= TOL32_STEP, err
    del q, qd0
    s.close()
    torch.cuda.empty_cache()
