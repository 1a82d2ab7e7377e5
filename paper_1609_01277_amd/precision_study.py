"""FP32 form against the FP64 form: Taylor-Green at 512^3, order 4, 2000 RK3 steps.

Both runs use the same initial state (the library's Taylor-Green initialiser, in
double, rounded to the state type) and the paper's time step for 512^3.  Every
`--every` steps the FP64 compensated diagnostics (kinetic energy, enstrophy,
conservation sums) of both states are taken; the JSON output has the per-sample
values and, per diagnostic, the largest and final relative error of FP32 against
FP64.  For the momentum sums, whose exact value is 0, the error is taken relative
to the mean |rho u_i| scale <|rho u|> = 1/(2 sqrt 2) of the initial field.
"""
import argparse
import json
import sys
import time

import numpy as np


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def run(dtype, n, order, steps, every):
    import torch

    import synth
    from paper_1609_01277_amd import DIAG_NAMES, Solver
    s = Solver(n, order=order, dtype=dtype, **synth.TGV)
    s.autotune()
    q, qt, dq = s.empty_state(), s.empty_state(), s.empty_state()
    s.tgv_init(q)
    dt = synth.tgv_dt(n)
    rows = []
    t0 = time.time()
    for k in range(0, steps + 1, every):
        d, code = s.diagnostics(q, check=False)
        rows.append([k * dt] + [d[nm] for nm in DIAG_NAMES] + [code])
        if k < steps:
            s.rk3_step(q, qt, dq, dt, every)
        if k % (10 * every) == 0:
            log("%s: step %d, %.1f s" % (dtype, k, time.time() - t0))
    torch.cuda.synchronize()
    sec = time.time() - t0
    del q, qt, dq
    s.close()
    torch.cuda.empty_cache()
    return np.array(rows), sec


def main(argv=None):
    import torch
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--order", type=int, default=4)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--every", type=int, default=10)
    ap.add_argument("--out", default="precision_study.json")
    args = ap.parse_args(argv)
    torch.cuda.set_device(0)
    from paper_1609_01277_amd import DIAG_NAMES
    r64, s64 = run("f64", args.n, args.order, args.steps, args.every)
    r32, s32 = run("f32", args.n, args.order, args.steps, args.every)
    scale = {"Ek": None, "enstrophy": None, "rho": None, "rhou": 1 / (2 * 2 ** 0.5), "rhov": 1 / (2 * 2 ** 0.5),
             "rhow": 1 / (2 * 2 ** 0.5), "rhoE": None}
    errs = {}
    for j, nm in enumerate(DIAG_NAMES):
        a, b = r32[:, 1 + j], r64[:, 1 + j]
        den = np.abs(b) if scale[nm] is None else scale[nm]
        e = np.abs(a - b) / den
        errs[nm] = {"max": float(np.max(e)), "final": float(e[-1])}
    out = {"n": args.n, "order": args.order, "steps": args.steps, "every": args.every,
           "seconds_f64": s64, "seconds_f32": s32, "relative_error_fp32_vs_fp64": errs,
           "t": r64[:, 0].tolist(), "f64": r64[:, 1:8].tolist(), "f32": r32[:, 1:8].tolist(),
           "status_f64": int(np.max(np.abs(r64[:, 8]))), "status_f32": int(np.max(np.abs(r32[:, 8])))}
    with open(args.out, "w") as f:
        json.dump(out, f)
    for nm, e in errs.items():
        log("%-10s max rel err %.3e, final %.3e" % (nm, e["max"], e["final"]))


if __name__ == "__main__":
    main()
