"""Every compiled launch variant and z-chunk of the fused stage kernel gives a bitwise
identical state (same arithmetic per point), and the autotuner keeps that property."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def _sbli():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a HIP device")
    import paper_1609_01277_amd as sbli
    return sbli, torch


CASES = [("f64", 4), ("f64", 8), ("f64", 6), ("f64", 2), ("f32", 4), ("f32", 8), ("f32", 6)]


@pytest.mark.parametrize("dtype,order", CASES)
def test_variants_bitwise_identical(dtype, order):
    sbli, torch = _sbli()
    n = (36, 20, 44)
    q0 = synth.random_conservative_state(n, seed=21, mom=0.3)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    s = sbli.Solver(n, order=order, dtype=dtype, **synth.TGV)
    nz = n[2]
    results = {}
    for v in range(len(s.variants())):
        for zc in (nz, 11, 5):
            s.set_tuning(v, zc)
            q = torch.from_numpy(q0).to(tdt).cuda()
            R = s.rhs(q)
            s.rk3_step(q, s.empty_state(), s.empty_state(), 1e-3, 2)
            results[(v, zc)] = (R.cpu().numpy(), q.cpu().numpy())
    ref = results[(0, nz)]
    for key, (R, q) in results.items():
        assert np.array_equal(R, ref[0]), ("rhs", key, s.variants()[key[0]])
        assert np.array_equal(q, ref[1]), ("rk3", key, s.variants()[key[0]])
    if dtype == "f64":
        p = oracle.Params(n=n, order=order, **synth.TGV)
        qo = oracle.rk3(q0, p, 1e-3, 2)
        mom = np.abs(qo[1:4]).max()
        for f in range(5):
            scale = mom if f in (1, 2, 3) else np.abs(qo[f]).max()
            assert np.abs(ref[1][f] - qo[f]).max() / scale <= 1e-12


@pytest.mark.parametrize("order", [4, 8])
def test_staged_form_bitwise_across_nested_runs(order):
    """nz = 100: the staged form's z-marching nested-field step runs 64 planes, then a
    run of 36 that starts inside the box; its residual and RK3 steps stay bitwise equal
    to the fused kernel's."""
    sbli, torch = _sbli()
    n = (20, 18, 100)
    q0 = synth.random_conservative_state(n, seed=22, mom=0.3)
    s = sbli.Solver(n, order=order, **synth.TGV)
    nv = len(s.variants())
    out = []
    for v in (0, nv - 1):                 # a fused variant, then the staged form
        s.set_tuning(v, n[2])
        q = torch.from_numpy(q0).cuda()
        R = s.rhs(q)
        s.rk3_step(q, s.empty_state(), s.empty_state(), 1e-3, 2)
        out.append((R.cpu().numpy(), q.cpu().numpy()))
    assert s.variants()[nv - 1] == (0, 0, 0, 0, 0, 0, 0)
    assert np.array_equal(out[0][0], out[1][0])
    assert np.array_equal(out[0][1], out[1][1])
    s.close()


def test_autotune_selects_valid_config(tmp_path):
    sbli, torch = _sbli()
    n = 48
    s = sbli.Solver(n, order=4, **synth.TGV)
    ent = s.autotune(reps=1, force=True, path=str(tmp_path / "cache.json"))
    v, zc = s.get_tuning()
    assert ent["variant"] == v and ent["zchunk"] == zc and 1 <= zc <= n
    assert ent["ms_per_step"] > 0
    again = s.autotune(reps=1, path=str(tmp_path / "cache.json"))
    assert again["cached"] and again["variant"] == v
    with pytest.raises(sbli.SbliError):
        s.set_tuning(99, 8)
    with pytest.raises(sbli.SbliError):
        s.set_tuning(0, n + 1)
