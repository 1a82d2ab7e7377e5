"""Learned-closure study: data from filtered fine solutions, training, a-posteriori test.

1. Fine Taylor-Green runs (256^3, FP64, order 4, dt 8.4625e-4) at Re in {800, 1600,
   3200} to t = 10.  At evenly spaced times the state q_f is box-filtered to 64^3
   (width 4 fine cells), together with its residual: the training pair is
   (F q_f, C* = F R_f(q_f) - R_c(F q_f)), R_c the coarse 64^3 FP32 residual.
   With --inputs coarse the input is instead the state q_c of the plain coarse
   solver run alongside from F q_f(0) (one coarse step per `ratio` fine steps), and
   the target C* = F R_f(q_f) - R_c(q_c): the network is trained on the states a
   coarse run produces, which are the states it meets once coupled.
2. Per-field standardisation from the pairs, Adam training of the closure network
   (BF16 MFMA kernels of the library) on the pairs.  With --aggregate K (coarse
   inputs), K more rounds follow: the fine and coarse runs are repeated with the
   trained closure coupled into the coarse run, the pairs (q_cc, F R_f(q_f) -
   R_c(q_cc)) are collected at the states that coupled run visits (R_c the plain
   coarse residual), and training continues on all pairs so far (dataset
   aggregation: the network learns the states its own feedback produces).
3. A-posteriori: coarse 64^3 FP32 runs (dt 3.385e-3) from F q_f(0) to t = 10 with
   and without the closure; filtered kinetic energy and enstrophy against those of
   F q_f(t) (the filtered fine solution is the reference for the error).

Every arithmetic step runs in libsbli's kernels; torch only holds device memory and
copies samples into batch buffers.  Writes one JSON file.
"""
import argparse
import json
import math
import sys
import time

import numpy as np


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def main(argv=None):
    import torch

    import synth
    from paper_1609_01277_amd import Solver
    from paper_1609_01277_amd import closure as cl

    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--out", default="closure_study.json")
    ap.add_argument("--nf", type=int, default=256)
    ap.add_argument("--ratio", type=int, default=4)
    ap.add_argument("--t-end", type=float, default=10.0)
    ap.add_argument("--res", default="800,1600,3200")
    ap.add_argument("--snapshots", type=int, default=2000)
    ap.add_argument("--epochs", type=int, default=16)
    ap.add_argument("--batch", type=int, default=4)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--seed", type=int, default=1609)
    ap.add_argument("--guard", type=float, default=2.0,
                    help="guard limit per field = guard * (largest |C*| of that field in the training set)")
    ap.add_argument("--diag-every", type=int, default=10, help="coarse steps between diagnostics")
    ap.add_argument("--hold-out", type=int, default=10,
                    help="every n-th snapshot is held out of training for the a-priori test")
    ap.add_argument("--inputs", choices=["filtered", "coarse"], default="filtered",
                    help="network inputs of the training pairs: the filtered fine state, or the state of "
                         "the plain coarse solver run alongside")
    ap.add_argument("--aggregate", type=int, default=0,
                    help="rounds of dataset aggregation (coarse inputs only): pairs from the closure-coupled "
                         "coarse run, then more training on all pairs")
    ap.add_argument("--aggregate-epochs", type=int, default=4, help="training epochs after each aggregation round")
    ap.add_argument("--noise", type=float, default=0.0,
                    help="input-noise injection: every training input is perturbed by Gaussian noise of this many "
                         "times its field's training-set standard deviation (the target stays that of the clean "
                         "input), so the network meets states off the training trajectories")
    ap.add_argument("--conservative", action="store_true",
                    help="after training, remove the box mean of every field of the closure term (the exact "
                         "term has none), so the coupled run keeps the totals of mass, momentum and energy")
    args = ap.parse_args(argv)
    if args.aggregate and args.inputs != "coarse":
        ap.error("--aggregate needs --inputs coarse")

    torch.cuda.set_device(0)
    nf, r = args.nf, args.ratio
    nc = nf // r
    Pc = nc ** 3
    dt_f = synth.DT64 * 64.0 / nf
    dt_c = dt_f * r
    res = [float(v) for v in args.res.split(",")]
    steps_f = int(round(args.t_end / dt_f))
    per_re = [args.snapshots // len(res) + (1 if i < args.snapshots % len(res) else 0) for i in range(len(res))]
    nrounds = 1 + args.aggregate
    X = torch.empty((args.snapshots * nrounds, 5, nc, nc, nc), dtype=torch.float32, device="cuda")
    Y = torch.empty_like(X)
    out = {"config": vars(args), "nf": nf, "nc": nc, "dt_fine": dt_f, "dt_coarse": dt_c, "fine_steps": steps_f}
    ref_diag = {}
    t0 = time.time()

    def collect(k, net=None):
        """Fine runs at every Re with a coarse run alongside (coupled to `net` when
        given); pairs from index k on.  Returns the next free index."""
        k_end = k + args.snapshots
        for ri, Re in enumerate(res):
            fine = Solver(nf, order=4, dtype="f64", Re=Re, Mach=0.1, Pr=0.71, gamma=1.4)
            fine.autotune()
            coarse = Solver(nc, order=4, dtype="f32", Re=Re, Mach=0.1, Pr=0.71, gamma=1.4)
            plain = Solver(nc, order=4, dtype="f32", Re=Re, Mach=0.1, Pr=0.71, gamma=1.4) if net else coarse
            q, qt, dq = fine.empty_state(), fine.empty_state(), fine.empty_state()
            fine.tgv_init(q)
            Rf = fine.empty_state()
            fq = torch.empty((5, nc, nc, nc), dtype=torch.float32, device="cuda")
            along = args.inputs == "coarse"
            if along:
                # snapshots where a coarse step ends, so both runs are at the same time
                snap_steps = sorted(set(r * int(round(i * steps_f / r / max(per_re[ri] - 1, 1)))
                                        for i in range(per_re[ri])))
                qc, qct, dqc = coarse.empty_state(), coarse.empty_state(), coarse.empty_state()
                cl.sbli_box_filter(q, nf, 5, r, qc)
                if net is not None:
                    cl.attach(coarse, net)
            else:
                snap_steps = sorted(set(int(round(i * steps_f / max(per_re[ri] - 1, 1))) for i in range(per_re[ri])))
            snap_set = set(snap_steps)
            diag_every_f = args.diag_every * r
            ek, en, times = [], [], []
            for step in range(steps_f + 1):
                if step in snap_set and k < k_end:
                    if along:
                        X[k].copy_(qc)
                    else:
                        cl.sbli_box_filter(q, nf, 5, r, X[k])
                    fine.rhs(q, Rf)
                    plain.rhs(X[k], Y[k])                          # plain R_c of the input state
                    cl.sbli_box_filter(Rf, nf, 5, r, Y[k], subtract=True)   # C* = F R_f - R_c(input)
                    k += 1
                if net is None and step % diag_every_f == 0:
                    cl.sbli_box_filter(q, nf, 5, r, fq)
                    d, _ = coarse.diagnostics(fq, check=False)
                    ek.append(d["Ek"])
                    en.append(d["enstrophy"])
                    times.append(step * dt_f)
                if step < steps_f:
                    fine.rk3_step(q, qt, dq, dt_f, 1)
                    if along and (step + 1) % r == 0:
                        coarse.rk3_step(qc, qct, dqc, dt_c, 1)
                if step % 2000 == 0:
                    log("Re %g: fine step %d / %d, %d snapshots, %.1f s" % (Re, step, steps_f, k, time.time() - t0))
            if net is None:
                ref_diag[Re] = {"t": times, "Ek": ek, "enstrophy": en}
            if along:
                if net is not None:
                    cl.attach(coarse, None)
                del qc, qct, dqc
            del q, qt, dq, Rf
            fine.close()
            coarse.close()
            if net is not None:
                plain.close()
            torch.cuda.empty_cache()
        return k

    k = collect(0)
    out["data_seconds"] = time.time() - t0
    nsnap = k
    out["snapshots"] = nsnap

    # ---- standardisation and training ----
    net = cl.ClosureNet(nc, args.batch)
    net.channel_stats(X[:nsnap], 0)
    net.channel_stats(Y[:nsnap], 1)
    st = net.get_stats()
    st[20:25] = args.guard * st[30:35]
    net.set_stats(st)
    out["stats"] = [float(v) for v in st]
    net.set_params(synth.closure_init_params(args.seed))
    rng = np.random.default_rng(args.seed)
    xb = torch.empty((args.batch, 5, nc, nc, nc), dtype=torch.float32, device="cuda")
    yb = torch.empty_like(xb)
    held = np.arange(0, nsnap, args.hold_out) if args.hold_out > 0 else np.zeros(0, dtype=int)
    noise_scale = torch.tensor(args.noise * st[5:10], dtype=torch.float32, device="cuda").view(1, 5, 1, 1, 1)
    noise_gen = torch.Generator(device="cuda")
    noise_gen.manual_seed(args.seed)
    flop_per_sample = 2 * Pc * 27 * (8 * 32 + 32 * 32 + 32 * 32) * 3   # fwd + bwd-data + bwd-weight, padded

    def train(train_idx, epochs):
        losses = []
        steps_per_epoch = len(train_idx) // args.batch
        for ep in range(epochs):
            perm = train_idx[rng.permutation(len(train_idx))]
            tot = 0.0
            for s_ in range(steps_per_epoch):
                idx = perm[s_ * args.batch:(s_ + 1) * args.batch]
                for j, i in enumerate(idx):
                    xb[j].copy_(X[int(i)])
                    yb[j].copy_(Y[int(i)])
                if args.noise > 0:
                    xb.add_(torch.randn(xb.shape, device="cuda", generator=noise_gen) * noise_scale)
                tot += net.train_step(xb, yb, args.lr)
            losses.append(tot / steps_per_epoch)
            log("epoch %d: mean loss %.5f (%.1f s)" % (ep, losses[-1], time.time() - t1))
        return losses, epochs * steps_per_epoch

    train_idx = np.setdiff1d(np.arange(nsnap), held)
    t1 = time.time()
    torch.cuda.synchronize()
    losses, nsteps_train = train(train_idx, args.epochs)
    torch.cuda.synchronize()
    train_s = time.time() - t1
    out["training"] = {"epoch_loss": losses, "seconds": train_s, "steps": nsteps_train,
                       "ms_per_step": 1e3 * train_s / max(nsteps_train, 1),
                       "padded_tflops_per_s": flop_per_sample * args.batch * nsteps_train / train_s / 1e12,
                       "note": "wall time per step includes host-side batch assembly and the loss read-back"}
    if args.conservative:
        net.set_conservative(True)
    # dataset aggregation: pairs at the states of the closure-coupled coarse run
    rounds = []
    for rd in range(args.aggregate):
        k0 = k
        k = collect(k, net)
        agg_idx = np.concatenate([train_idx, np.arange(nsnap, k)])
        t1 = time.time()
        l_, n_ = train(agg_idx, args.aggregate_epochs)
        torch.cuda.synchronize()
        rounds.append({"pairs_added": int(k - k0), "pairs_total": int(len(agg_idx)), "epoch_loss": l_,
                       "seconds": time.time() - t1})
        log("aggregation round %d: %d pairs added, %d in training" % (rd + 1, k - k0, len(agg_idx)))
    if rounds:
        # the guard limits follow the pairs trained on (the standardisation stays)
        net.channel_stats(Y[:k], 1)
        st_all = net.get_stats()
        st[20:25] = args.guard * st_all[30:35]
        st[30:35] = st_all[30:35]
        net.set_stats(st)
        out["aggregation"] = rounds
        out["stats_after_aggregation"] = [float(v) for v in st]
    # time the network kernels alone on one batch (no host work in the loop)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        net.gradients(xb, yb)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 10
    out["training"]["fwd_bwd_ms_per_batch"] = ms
    out["training"]["fwd_bwd_padded_tflops_per_s"] = flop_per_sample * args.batch / (ms * 1e-3) / 1e12

    # ---- a-priori: the closure term on held-out snapshots ----
    # relative L2 error of the predicted closure term against C*, per field; the
    # method without the closure predicts C = 0, i.e. a relative error of 1
    num = np.zeros(5)
    den = np.zeros(5)
    pred = torch.empty((1, 5, nc, nc, nc), dtype=torch.float32, device="cuda")
    for i in held:
        net.forward(X[int(i)][None], pred)
        d = (pred[0].double() - Y[int(i)].double()).reshape(5, -1)
        num += (d * d).sum(dim=1).cpu().numpy()
        den += (Y[int(i)].double().reshape(5, -1) ** 2).sum(dim=1).cpu().numpy()
    if len(held):
        rel = np.sqrt(num / np.maximum(den, 1e-300))
        out["a_priori"] = {"held_out_snapshots": int(len(held)),
                           "rel_l2_err_per_field": [float(v) for v in rel],
                           "rel_l2_err_all": float(math.sqrt(num.sum() / max(den.sum(), 1e-300))),
                           "rel_l2_err_without_closure": 1.0}
        log("a-priori (held-out): relative L2 error per field %s, all %.4f (1 without closure)" % (
            np.array2string(rel, precision=4), out["a_priori"]["rel_l2_err_all"]))

    # ---- a-posteriori: coarse runs with and without the closure ----
    steps_c = int(round(args.t_end / dt_c))
    post = {}
    for Re in res:
        res_run = {}
        for mode in ("plain", "closure"):
            s = Solver(nc, order=4, dtype="f32", Re=Re, Mach=0.1, Pr=0.71, gamma=1.4)
            fine = Solver(nf, order=4, dtype="f64", Re=Re, Mach=0.1, Pr=0.71, gamma=1.4)
            qf = fine.tgv_init(fine.empty_state())
            q = s.empty_state()
            cl.sbli_box_filter(qf, nf, 5, r, q)
            del qf
            fine.close()
            if mode == "closure":
                cl.attach(s, net)
            qt, dq = s.empty_state(), s.empty_state()
            ek, en, mass, energy = [], [], [], []
            ratio = []          # per diagnostic step: per-field max |C| / guard limit
            cmean = []          # per diagnostic step: per-field |box mean of C| / max |C|
            limit = torch.tensor(st[20:25], dtype=torch.float32, device="cuda")
            t2 = time.time()
            for step in range(steps_c + 1):
                if step % args.diag_every == 0:
                    d, code = s.diagnostics(q, check=False)
                    ek.append(d["Ek"])
                    en.append(d["enstrophy"])
                    mass.append(d["rho"])
                    energy.append(d["rhoE"])
                    if mode == "closure":
                        net.forward(q[None], pred)
                        amax = pred[0].abs().reshape(5, -1).amax(dim=1)
                        ratio.append((amax / limit).cpu().tolist())
                        cmean.append((pred[0].double().reshape(5, -1).mean(dim=1).abs() / amax.double()).cpu().tolist())
                if step < steps_c:
                    s.rk3_step(q, qt, dq, dt_c, 1)
            torch.cuda.synchronize()
            refd = ref_diag[Re]
            m = min(len(ek), len(refd["Ek"]))
            e_ek = np.abs(np.array(ek[:m]) - np.array(refd["Ek"][:m])) / np.max(np.abs(refd["Ek"][:m]))
            e_en = np.abs(np.array(en[:m]) - np.array(refd["enstrophy"][:m])) / np.max(np.abs(refd["enstrophy"][:m]))
            entry = {"Ek_err_max": float(e_ek.max()), "Ek_err_rms": float(math.sqrt(np.mean(e_ek ** 2))),
                     "enstrophy_err_max": float(e_en.max()), "enstrophy_err_rms": float(math.sqrt(np.mean(e_en ** 2))),
                     # largest relative change of the box totals of mass and total energy over the run
                     "mass_drift_max": float(np.max(np.abs(np.array(mass) / mass[0] - 1.0))),
                     "energy_drift_max": float(np.max(np.abs(np.array(energy) / energy[0] - 1.0))),
                     "seconds": time.time() - t2, "Ek": ek, "enstrophy": en}
            if mode == "closure":
                entry["guard_accepted_rejected"] = list(cl.counts(s))
                r_ = np.array(ratio)
                entry["guard_ratio_max_per_field"] = r_.max(axis=0).tolist()
                entry["closure_mean_over_max_per_field"] = np.array(cmean).max(axis=0).tolist()
                over = np.nonzero(r_.max(axis=1) > 1.0)[0]
                entry["guard_first_exceed_t"] = float(over[0] * args.diag_every * dt_c) if len(over) else None
                log("Re %g closure: guard accepted %d rejected %d; max |C|/limit per field %s; first exceeded at t = %s" % (
                    Re, entry["guard_accepted_rejected"][0], entry["guard_accepted_rejected"][1],
                    np.array2string(r_.max(axis=0), precision=3), entry["guard_first_exceed_t"]))
                cl.attach(s, None)
            res_run[mode] = entry
            log("Re %g %s: Ek err max %.4f rms %.4f; enstrophy err max %.4f rms %.4f; mass drift %.2e, energy drift %.2e" % (
                Re, mode, entry["Ek_err_max"], entry["Ek_err_rms"], entry["enstrophy_err_max"],
                entry["enstrophy_err_rms"], entry["mass_drift_max"], entry["energy_drift_max"]))
            s.close()
        res_run["reference"] = ref_diag[Re]
        post[str(Re)] = res_run
    out["a_posteriori"] = post
    with open(args.out, "w") as f:
        json.dump(out, f)
    log("wrote", args.out)


if __name__ == "__main__":
    main()
