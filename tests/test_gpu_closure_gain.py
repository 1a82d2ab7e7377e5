"""What the trained closure gains over the method without it (small configuration of
the closure study: 128^3 FP64 fine runs filtered to 32^3, Re 1600, t in [0, 2]).

A-priori: on snapshots held out of training, the network's closure term is closer to
the filtered-fine target C* = F R_f - R_c(F q_f) than the method without closure
(which predicts 0, relative error 1).  A-posteriori: the coarse run with the closure
stays finite, the guard accepts the network's terms, and the filtered kinetic energy
error against the filtered fine solution is reported next to the plain coarse run's.
"""
import json
import math

import pytest

pytestmark = pytest.mark.gpu


def test_trained_closure_beats_plain_coarse_operator(tmp_path):
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a HIP device")
    from paper_1609_01277_amd import closure_study
    out = tmp_path / "closure_small.json"
    closure_study.main(["--nf", "128", "--t-end", "2", "--res", "1600", "--snapshots", "200",
                        "--epochs", "12", "--hold-out", "10", "--out", str(out)])
    d = json.loads(out.read_text())
    ap = d["a_priori"]
    print("a-priori relative L2 error per field:", ap["rel_l2_err_per_field"], "all:", ap["rel_l2_err_all"])
    assert ap["held_out_snapshots"] == 20
    assert ap["rel_l2_err_all"] < 0.9
    post = d["a_posteriori"]["1600.0"]
    plain, clos = post["plain"], post["closure"]
    print("Ek error max: plain %.4g, closure %.4g" % (plain["Ek_err_max"], clos["Ek_err_max"]))
    acc, rej = clos["guard_accepted_rejected"]
    assert acc > 0
    for e in (plain, clos):
        assert all(math.isfinite(v) for v in e["Ek"] + e["enstrophy"])
