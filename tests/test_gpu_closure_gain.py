"""What the trained closure gains over the method without it (small configuration of
the closure study: 128^3 FP64 fine runs filtered to 32^3, Re 1600, t in [0, 2]).

Three ways of making training pairs, each followed by coupled (a-posteriori) coarse runs
with and without the closure, judged against the filtered fine solution:
- inputs the filtered fine state F q_f (target F R_f - R_c(F q_f));
- inputs the state of the plain coarse solver run alongside, q_c (target
  F R_f - R_c(q_c)): the network then trains on the kind of state it meets when
  coupled;
- filtered inputs with input-noise injection (each training input perturbed by
  Gaussian noise of 0.1 times its field's standard deviation, clean targets).
For each: the guard accepts (almost) every evaluation, and the maximum over time of the
filtered kinetic-energy and enstrophy errors is below the plain coarse run's.  The
filtered-input network also beats the method without closure a-priori (held-out
snapshots; relative L2 error of the closure term, 1 without closure).
"""
import json
import math

import pytest

pytestmark = pytest.mark.gpu


def _run(tmp_path, inputs, noise):
    from paper_1609_01277_amd import closure_study
    out = tmp_path / ("closure_small_%s_%g.json" % (inputs, noise))
    closure_study.main(["--nf", "128", "--t-end", "2", "--res", "1600", "--snapshots", "200",
                        "--epochs", "12", "--hold-out", "10", "--inputs", inputs, "--noise", str(noise),
                        "--out", str(out)])
    return json.loads(out.read_text())


@pytest.mark.parametrize("inputs,noise", [("filtered", 0.0), ("coarse", 0.0), ("filtered", 0.1)])
def test_trained_closure_beats_plain_coarse_run(tmp_path, inputs, noise):
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a HIP device")
    d = _run(tmp_path, inputs, noise)
    ap = d["a_priori"]
    post = d["a_posteriori"]["1600.0"]
    plain, clos = post["plain"], post["closure"]
    acc, rej = clos["guard_accepted_rejected"]
    print("inputs %s, noise %g: a-priori relative L2 error %.4f; a-posteriori max error, plain vs closure: "
          "Ek %.4g vs %.4g, enstrophy %.4g vs %.4g; guard accepted %d, rejected %d" % (
              inputs, noise, ap["rel_l2_err_all"], plain["Ek_err_max"], clos["Ek_err_max"],
              plain["enstrophy_err_max"], clos["enstrophy_err_max"], acc, rej))
    for e in (plain, clos):
        assert all(math.isfinite(v) for v in e["Ek"] + e["enstrophy"])
    assert acc >= 0.9 * (acc + rej)
    assert clos["Ek_err_max"] < plain["Ek_err_max"]
    assert clos["enstrophy_err_max"] < plain["enstrophy_err_max"]
    if inputs == "filtered":
        assert ap["held_out_snapshots"] == 20
        assert ap["rel_l2_err_all"] < 0.5
