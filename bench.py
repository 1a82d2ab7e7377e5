#!/usr/bin/env python3
"""Throughput of the fused Navier-Stokes RK3 step on one MI355X.

Workload: the Taylor-Green vortex of the OpenSBLI paper (Sec. "3D Taylor-Green
vortex") at 512^3, FP64, 4th-order central differences, low-storage RK3 with the
paper's time step for that grid (3.385e-3 at 64^3, halved per doubling).  A step
is one pass of the whole hot path: three fused residual + RK-update stages over
the full grid.  The state starts resident in HBM.

The line's value is the median of three timed runs of --steps steps.  Prints ONE JSON
line on stdout.  Extra measurements (FP32 state, orders 8 and 12, 256^3, the grid study's
200-step schedule with diagnostics every 10 steps, the 64-box ensemble and its FP32 error,
the closure network's kernels) and the CPU oracle baseline are attached to the same line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E peak, GB/s
WORDS_PER_POINT_STEP = 50      # algorithmic words per point per RK3 step (15 + 20 + 15)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


KERNEL_SOURCES = ("kernels_stage_fused.h", "stage_variants.h", "sbli_common.h")
COUNTERS_FILE = os.path.join(ROOT, "profiles", "fused_stage_counters.json")


def kernel_source_hash():
    """sha256 over the sources of the fused stage kernel."""
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1609_01277_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def counted_traffic(n, order, dtype, tuning):
    """HBM bytes per stage launch from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE
    summary, scaled by the plain-copy calibration; None when that summary was taken
    on other kernel sources or another workload / launch configuration."""
    try:
        with open(COUNTERS_FILE) as f:
            c = json.load(f)
    except (OSError, ValueError):
        return None
    if c.get("kernel_source_sha256") != kernel_source_hash():
        return None
    if (c.get("n"), c.get("order"), c.get("dtype")) != (n, order, dtype):
        return None
    if tuning is None or c.get("tile") != tuning.get("tile") or c.get("zchunk") != tuning.get("zchunk"):
        return None
    return 1024.0 * (c["fetch_kib_per_dispatch"] * c["copy_fetch_factor"]
                     + c["write_kib_per_dispatch"] * c["copy_write_factor"])


def measure(sbli, torch, n, order, dtype, steps, warmup, runs=3):
    """Time `runs` runs of `steps` RK3 steps after `warmup` (HIP events on the solver's
    stream, state resident in HBM) and keep the median run; returns a dict of results."""
    import synth
    s = sbli.Solver(n, order=order, dtype=dtype, **synth.TGV)
    tune = s.autotune(reps=2)
    q, qt, dq = s.empty_state(), s.empty_state(), s.empty_state()
    s.tgv_init(q)
    dt = synth.tgv_dt(n)
    stream = torch.cuda.current_stream()
    if warmup:
        s.rk3_step(q, qt, dq, dt, warmup)
    torch.cuda.synchronize()
    times = []
    for _ in range(runs):
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        s.rk3_step(q, qt, dq, dt, steps)
        ev1.record(stream)
        torch.cuda.synchronize()
        times.append(ev0.elapsed_time(ev1))
    ms = sorted(times)[len(times) // 2]
    diag, code = s.diagnostics(q, check=False)
    P = n ** 3
    word = 8 if dtype == "f64" else 4
    launches = 3 * steps
    avg_launch_ms = ms / launches
    bytes_per_launch = WORDS_PER_POINT_STEP * word * P / 3.0
    achieved = bytes_per_launch / (avg_launch_ms * 1e-3) / 1e9
    del q, qt, dq
    s.close()
    torch.cuda.empty_cache()
    return dict(n=n, order=order, dtype=dtype, steps=steps, ms=ms, ms_per_step=ms / steps,
                run_ms=times, value=P * steps / (ms * 1e-3) / 1e6, avg_launch_ms=avg_launch_ms,
                bytes_per_launch=bytes_per_launch, achieved_gbs=achieved,
                frac=achieved / HBM_PEAK_GBS, diag_status=code, Ek=diag["Ek"],
                enstrophy=diag["enstrophy"], tuning=tune)


def measure_schedule(sbli, torch, n, order, steps=200, every=10):
    """The Taylor-Green throughput schedule of the paper's grid study at one size and
    order: `steps` RK3 steps from the initial state with kinetic energy and enstrophy
    taken every `every` steps (and at the start), timed end to end on the host clock
    with the diagnostics in it; also the stepping alone (HIP events)."""
    import synth
    s = sbli.Solver(n, order=order, dtype="f64", **synth.TGV)
    s.autotune(reps=2)
    q, qt, dq = s.empty_state(), s.empty_state(), s.empty_state()
    dt = synth.tgv_dt(n)
    stream = torch.cuda.current_stream()
    s.tgv_init(q)
    s.rk3_step(q, qt, dq, dt, 1)          # warm-up step, then start again from t = 0
    s.tgv_init(q)
    torch.cuda.synchronize()
    samples = []
    step_ms = 0.0
    t0 = time.perf_counter()
    for k in range(0, steps + 1, every):
        d, code = s.diagnostics(q, check=False)
        samples.append((k * dt, d["Ek"], d["enstrophy"]))
        if k < steps:
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            s.rk3_step(q, qt, dq, dt, every)
            e1.record(stream)
            e1.synchronize()
            step_ms += e0.elapsed_time(e1)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    del q, qt, dq
    s.close()
    torch.cuda.empty_cache()
    P = n ** 3
    return {"n": n, "order": order, "steps": steps, "diagnostics_every": every,
            "value_with_diagnostics": P * steps / wall / 1e6,
            "value_stepping_only": P * steps / (step_ms * 1e-3) / 1e6,
            "wall_s": wall, "stepping_ms": step_ms, "samples_t_Ek_enstrophy": samples,
            "unit": "Mpoint-RK3-steps/s"}


def measure_batch(sbli, torch, steps):
    """64-box FP32 ensemble (seed 1609): one hipGraph replay of `steps` steps vs the
    same steps box by box (3 launches per box per step)."""
    import synth
    b = sbli.Batch(synth.batch_instances(), order=4, dtype="f32")
    tune_ms = b.autotune(reps=2)
    q, qt, dq = b.tgv_init(b.empty_state()), b.empty_state(), b.empty_state()
    pts = b.points()
    stream = torch.cuda.current_stream()
    b.capture(q, qt, dq, steps)
    b.launch()                      # warm-up replay
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    b.launch()
    e1.record(stream)
    torch.cuda.synchronize()
    ms_graph = e0.elapsed_time(e1)
    b.step_sequential(q, qt, dq, 1)
    torch.cuda.synchronize()
    e0.record(stream)
    b.step_sequential(q, qt, dq, steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_seq = e0.elapsed_time(e1)
    diags, code = b.diagnostics(q, check=False)
    v, zmax = b.get_tuning()
    # error of the FP32 form: the same ensemble and steps from the initial state in
    # FP32 and in FP64, per-box kinetic energy and enstrophy (FP64 sums of both)
    b.tgv_init(q)
    b.step(q, qt, dq, steps)
    d32, _ = b.diagnostics(q, check=False)
    del q, qt, dq
    b.close()
    b64 = sbli.Batch(synth.batch_instances(), order=4, dtype="f64")
    q, qt, dq = b64.tgv_init(b64.empty_state()), b64.empty_state(), b64.empty_state()
    b64.step(q, qt, dq, steps)
    d64, _ = b64.diagnostics(q, check=False)
    del q, qt, dq
    b64.close()
    torch.cuda.empty_cache()
    rel = lambda k: max(abs(d32[i][k] - d64[i][k]) / abs(d64[i][k]) for i in range(len(d64)))
    return {"boxes": 64, "points": pts, "steps": steps,
            "graph_value": pts * steps / (ms_graph * 1e-3) / 1e6,
            "sequential_value": pts * steps / (ms_seq * 1e-3) / 1e6,
            "speedup": ms_seq / ms_graph, "graph_ms": ms_graph, "sequential_ms": ms_seq,
            "unit": "Mpoint-RK3-steps/s", "variant": v, "zmax": zmax, "status": code,
            "fp32_vs_fp64_after_steps": {"Ek_max_rel_err": rel(0), "enstrophy_max_rel_err": rel(1),
                                          "mean_rho_max_rel_err": rel(2), "mean_rhoE_max_rel_err": rel(6)}}


def measure_closure(torch, n=64, batch=4, reps=10):
    """The learned closure's BF16-MFMA kernels at the coarse grid: forward + backward
    (data and weight gradients) of a batch, and the forward of one sample."""
    import numpy as np
    import synth
    from paper_1609_01277_amd import closure
    net = closure.ClosureNet(n, batch)
    net.set_params(synth.closure_init_params(1609))
    st = np.zeros(closure.N_STATS, dtype=np.float32)
    st[5:10] = 1.0
    st[15:20] = 1.0
    st[20:25] = 1e30
    net.set_stats(st)
    g = torch.Generator(device="cuda").manual_seed(1609)
    x = torch.randn((batch, 5, n, n, n), device="cuda", generator=g)
    y = torch.randn((batch, 5, n, n, n), device="cuda", generator=g)
    net.gradients(x, y)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        net.gradients(x, y)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_train = e0.elapsed_time(e1) / reps
    out = torch.empty((1, 5, n, n, n), device="cuda")
    net.forward(x[:1], out)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(reps):
        net.forward(x[:1], out)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_fwd = e0.elapsed_time(e1) / reps
    net.close()
    # Algorithmic work per point (2 flops per multiply-add, 27 taps): the forward pass of
    # the 5-32-32-5 network (1,344 MACs per tap), the weight gradients of all three layers
    # (the same), and the data gradients of layers 3 and 2 (the input needs none).
    fwd = 2 * 27 * (5 * 32 + 32 * 32 + 32 * 5)
    train = 2 * fwd + 2 * 27 * (32 * 5 + 32 * 32)
    P = n ** 3
    tf_train = train * P * batch / (ms_train * 1e-3) / 1e12
    tf_fwd = fwd * P / (ms_fwd * 1e-3) / 1e12
    # what the MFMA kernels execute, channels padded to 8 / 32 and all three data gradients
    padded = 3 * 2 * 27 * (8 * 32 + 32 * 32 + 32 * 32)
    return {"grid": n, "batch": batch, "fwd_bwd_ms": ms_train, "fwd_bwd_tflops": tf_train,
            "flop_per_point_fwd_bwd": train, "forward_ms_1_sample": ms_fwd, "forward_tflops": tf_fwd,
            "flop_per_point_fwd": fwd, "bf16_dense_peak_tflops": 2500.0, "frac_fwd_bwd": tf_train / 2500.0,
            "fwd_bwd_padded_tflops": padded * P * batch / (ms_train * 1e-3) / 1e12}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(n=256, steps=3, n1=128):
    """The FP64 oracle, as it stands, on the host: `steps` RK3 steps of the Taylor-Green
    state at n^3 on all host threads for orders 4 and 8, and one step at n1^3 on one
    thread (order 4)."""
    import oracle
    import synth

    def run(nn, order, k):
        p = oracle.Params(n=(nn, nn, nn), order=order, **synth.TGV)
        q = oracle.tgv_init(p)
        t0 = time.perf_counter()
        oracle.rk3(q, p, synth.tgv_dt(nn), k)
        return time.perf_counter() - t0

    threads = oracle.num_threads()
    t4 = run(n, 4, steps)
    t8 = run(n, 8, steps)
    oracle.set_num_threads(1)
    try:
        t1 = run(n1, 4, 1)
    finally:
        oracle.set_num_threads(threads)
    return {"value": steps * n ** 3 / t4 / 1e6, "unit": "Mpoint-RK3-steps/s", "cores": threads,
            "kind": "oracle", "cpu_model": cpu_model(),
            "order8_value": steps * n ** 3 / t8 / 1e6,
            "single_thread_value": n1 ** 3 / t1 / 1e6,
            "sample": "whole-array C oracle (FP64, OpenMP over z-planes) on the Taylor-Green state: %d RK3 "
                      "steps at %d^3 on %d threads, order 4 (%.1f s; value) and order 8 (%.1f s; order8_value); "
                      "1 step at %d^3, order 4, on 1 thread (%.1f s; single_thread_value)"
                      % (steps, n, threads, t4, t8, n1, t1)}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--order", type=int, default=4)
    ap.add_argument("--dtype", default="f64", choices=["f64", "f32"])
    ap.add_argument("--no-extra", action="store_true", help="skip the FP32, order-8 and order-12 lines")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-n", type=int, default=256)
    ap.add_argument("--closure-only", action="store_true",
                    help="only time the learned closure's kernels (64^3, batch 4) and exit")
    ap.add_argument("--batch-only", action="store_true",
                    help="only time the 64-box FP32 ensemble (graph replay against box-by-box stepping) and exit")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run 5 device-to-device copies of MIB MiB (HBM counter calibration) and exit")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this library has no multi-GPU path "
              "(requested --gpus %d, WORLD_SIZE %d)" % (args.gpus, world), file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a HIP device", file=sys.stderr)
        sys.exit(2)
    torch.cuda.set_device(0)
    if args.calibrate_copy:
        # A plain copy of known size: its FETCH_SIZE / WRITE_SIZE counters give the
        # factor between counted and true HBM bytes.
        n = args.calibrate_copy * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(5):
            dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 5
        # bytes read plus bytes written per copy, over its average duration
        log("copied %d MiB x 5: %.3f ms per copy, %.0f GB/s read + write" % (
            args.calibrate_copy, ms, 2 * n * 8 / (ms * 1e-3) / 1e9))
        # streaming reads alone (a sum) and writes alone (a fill) of the same size
        for name, op in (("read (sum)", lambda: src.sum()), ("write (fill)", lambda: dst.fill_(2.0))):
            op()
            e0.record()
            for _ in range(5):
                op()
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / 5
            log("%s of %d MiB: %.3f ms, %.0f GB/s" % (name, args.calibrate_copy, ms, n * 8 / (ms * 1e-3) / 1e9))
        return
    from paper_1609_01277_amd import build as libbuild
    if not libbuild.is_current():
        # missing, or built from other sources than those in the tree
        import __graft_entry__
        __graft_entry__.build()
    import paper_1609_01277_amd as sbli

    if args.closure_only:
        print(json.dumps(measure_closure(torch)), flush=True)
        return
    if args.batch_only:
        print(json.dumps(measure_batch(sbli, torch, args.steps)), flush=True)
        return
    log("main: TGV %d^3 %s order %d, %d steps after %d warm-up" % (args.n, args.dtype, args.order,
                                                                  args.steps, args.warmup))
    main_r = measure(sbli, torch, args.n, args.order, args.dtype, args.steps, args.warmup)
    log("main: %.1f Mpt-steps/s, %.3f ms/step, %.0f GB/s (%.1f%% of HBM peak)" % (
        main_r["value"], main_r["ms_per_step"], main_r["achieved_gbs"], 100 * main_r["frac"]))

    extra = {}
    if not args.no_extra:
        for (dt_, order) in (("f32", args.order), ("f64", 8), ("f64", 12)):
            if dt_ == args.dtype and order == args.order:
                continue
            r = measure(sbli, torch, args.n, order, dt_, args.steps, args.warmup)
            key = "%s_order%d" % (dt_, order)
            extra[key] = {k: r[k] for k in ("value", "ms_per_step", "achieved_gbs", "frac", "tuning")}
            log("extra %s: %.1f Mpt-steps/s, %.0f GB/s (%.1f%%)" % (key, r["value"], r["achieved_gbs"],
                                                                    100 * r["frac"]))

    if not args.no_extra:
        for (nn, order) in ((256, 4), (256, 8)):
            r = measure(sbli, torch, nn, order, "f64", args.steps, args.warmup)
            key = "f64_order%d_%dcube" % (order, nn)
            extra[key] = {k: r[k] for k in ("value", "ms_per_step", "achieved_gbs", "frac", "tuning")}
            log("extra %s: %.1f Mpt-steps/s (%.1f%%)" % (key, r["value"], 100 * r["frac"]))
        # the grid study's schedule: 200 steps, kinetic energy and enstrophy every 10
        for (nn, order) in ((512, 4), (512, 8), (256, 4), (256, 8)):
            r = measure_schedule(sbli, torch, nn, order)
            extra["schedule_f64_order%d_%dcube" % (order, nn)] = r
            log("extra schedule %d^3 order %d: %.1f Mpt-steps/s with diagnostics every 10 steps "
                "(%.1f stepping only)" % (nn, order, r["value_with_diagnostics"], r["value_stepping_only"]))

    if not args.no_extra:
        rb = measure_batch(sbli, torch, 100)
        extra["batched_f32_order4_64boxes"] = rb
        log("extra batched: graph %.1f vs sequential %.1f Mpt-steps/s (x%.2f); FP32 vs FP64 after 100 "
            "steps: Ek %.2e, enstrophy %.2e" % (rb["graph_value"], rb["sequential_value"], rb["speedup"],
                                                 rb["fp32_vs_fp64_after_steps"]["Ek_max_rel_err"],
                                                 rb["fp32_vs_fp64_after_steps"]["enstrophy_max_rel_err"]))

    if not args.no_extra:
        rc = measure_closure(torch)
        extra["closure_bf16_64cube"] = rc
        log("extra closure: fwd+bwd batch 4 %.2f ms (%.1f TFLOP/s algorithmic, %.1f %% of BF16 dense), "
            "forward %.2f ms" % (rc["fwd_bwd_ms"], rc["fwd_bwd_tflops"], 100 * rc["frac_fwd_bwd"],
                                 rc["forward_ms_1_sample"]))

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline: oracle, 3 steps at %d^3 (orders 4, 8), 1 step at 128^3 on one thread" % args.cpu_n)
        cpu = cpu_baseline(args.cpu_n)
        log("cpu baseline: %.2f Mpt-steps/s on %d threads (%s); order 8 %.2f; one thread %.3f" % (
            cpu["value"], cpu["cores"], cpu["cpu_model"], cpu["order8_value"], cpu["single_thread_value"]))

    word = 8 if args.dtype == "f64" else 4
    line = {
        "metric": "Mpoint-RK3-steps/s, 4th-order TGV 512^3 FP64 vs FP32; % of HBM roofline",
        "value": main_r["value"],
        "unit": "Mpoint-RK3-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_r["ms_per_step"],
        "timed_runs_ms": main_r["run_ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic (analytic Taylor-Green initial state)",
        "config": {"workload": "Taylor-Green vortex %d^3, order %d, %s state, low-storage RK3, dt %.6g"
                               % (args.n, args.order, args.dtype.upper(), 64 * 3.385e-3 / args.n),
                   "n": args.n, "order": args.order, "points": args.n ** 3},
        "roofline": {"bound": "hbm", "achieved": main_r["achieved_gbs"], "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": main_r["frac"],
                     "traffic": counted_traffic(args.n, args.order, args.dtype, main_r["tuning"]),
                     "kernel": "RK3 stage (residual + update), all launches of the timed region",
                     "algorithmic_bytes_per_launch": main_r["bytes_per_launch"],
                     "avg_launch_ms": main_r["avg_launch_ms"],
                     "words_per_point_step": WORDS_PER_POINT_STEP, "word_bytes": word,
                     "launch": main_r["tuning"]},
        "cpu_baseline": cpu,
        "extra": extra,
        "diagnostics_after_run": {"Ek": main_r["Ek"], "enstrophy": main_r["enstrophy"],
                                  "status": main_r["diag_status"]},
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
