#!/usr/bin/env python3
"""Benchmark: SD DOF-updates/s of the SSP-RK3 spectral-difference solver on
one MI355X (mixed FP32/FP64 path, checked against the FP64 plain path on the
same run), with the dominant kernel's HBM roofline and the CPU oracle beside
it.

One step = one full SSP-RK3 step (three residual evaluations with the fused
stage update) over every solution point of the workload; DOFs = E N^3.  The
default workload is the 331,776-hex N = 4 Sun-like shell (21.2M DOFs), the
single-GPU stand-in at the paper's production scale.  Inputs are synthetic
and seeded: a cubed-sphere shell, the polytropic background and a seeded
entropy perturbation.

Timing: W untimed warm-up steps, then R repeats of K timed steps, each
bracketed by device synchronisation, with per-kernel event timing off; the
value is the median repeat.  One further K-step run with per-launch HIP-event
timing (on the launch stream) gives the kernels' average launch durations
for the roofline; it is not part of the value.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--repeats R] [--workload NAME]

Prints one JSON line.
"""
import argparse
import json
import os
import statistics
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "SD DOF-updates/s, mixed vs FP64 plain at ≤1e-6 rel err; % HBM roofline"
HBM_PEAK_GBS = 8000.0
# MI355X vector peaks: 256 CUs x 4 SIMDs x 2.4 GHz; FP32 157.3 TFLOP/s with
# packed FP32 (the library is built without packed FP32, so its own ceiling
# is the FP64-rate 78.6); FP64 78.6 TFLOP/s
ALU_PEAK_TFLOPS = {"mixed": 157.3, "fp64": 78.6}

# Algorithmic HBM bytes per DOF-update (one SSP-RK3 step of one solution
# point), the operation-count model of the hot path: 320 B of FP64 state
# (5 reads + 3 writes of 40 B), the 20 node coordinates and the face
# connectivity once per element and stage; the mixed path adds per stage the
# FP32 background residual, rho0 and p0 at every point and the background
# face jump with its wave speed at every face point.
ALG_BYTES_PER_DOF_UPDATE = {"fp64": {3: 379.0, 4: 345.0, 6: 327.0},
                            "mixed": {3: 472.0, 4: 445.0}}


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def alg_bytes_per_stage_point(N, precision):
    """Algorithmic bytes per solution point and residual stage (a third of
    the per-DOF-update figure)."""
    return ALG_BYTES_PER_DOF_UPDATE[precision][N] / 3.0


def kernel_source_sha():
    import hashlib
    h = hashlib.sha256()
    for f in ("sd_kernels.hip", "sd_mixed.hip", "sd_common.hpp", "physics.hpp", "launch.hpp"):
        with open(os.path.join(ROOT, "paper_1503_00834_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload, precision, kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, if it was taken on the current kernel sources (else None)."""
    name = os.path.join(ROOT, "profiles", "sd_%s_%s.md" % (precision, workload))
    if not os.path.exists(name):
        return None
    vals = {}
    with open(name) as f:
        for line in f:
            line = line.strip()
            for key in ("kernel:", "source_sha256:", "traffic_bytes_per_launch:"):
                if line.startswith(key):
                    vals[key[:-1]] = line.split(":", 1)[1].strip()
    if vals.get("source_sha256") != kernel_source_sha() or vals.get("kernel") != kernel:
        return None
    try:
        return float(vals["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def alg_flops_per_stage_point(N):
    """Algorithmic flops per solution point and residual stage (operation
    count of the method, +-30 %): the line operators (interpolation of 5
    values, differentiation of 5, interpolation of 15 gradients, divergence
    of 5 fluxes) take 90 (N+1) multiply-adds per point; the pointwise
    inviscid + viscous fluxes about 150 flops per flux point, of which there
    are 3 (N+1)/N per solution point; the face fluxes, the source and the
    stage update a few tens more.  Per SSP-RK3 step this is about 4.7k
    flops per point at N = 3 and 5.0k at N = 4."""
    per_step = {2: 4.4e3, 3: 4.7e3, 4: 5.0e3, 5: 5.4e3, 6: 5.9e3}[N]
    return per_step / 3.0


def closure_leg(panel_n=32, radial_n=16):
    """The learned closure on the closure-run shell (6 x 32 x 32 x 16 =
    98,304 hexes): order-3 steps with and without the fused bfloat16
    network, and the resolved order-6 run on the same mesh, per unit
    simulated time.  The network's matrix-core rate is its algorithmic
    flops (2 (20*64 + 64*64 + 64*15) = 12,672 per point) over the extra
    time its pass adds to the first pass of a stage."""
    from paper_1503_00834_amd import closure
    c = closure.cost_per_time(panel_n, radial_n, kernel_times=True)
    g_cl = c["closure"]["kernel_ms_per_launch"]["pass1"]
    g_pl = c["plain"]["kernel_ms_per_launch"]["pass1"]
    flops = 12672.0 * c["closure"]["points"]
    dt_mlp = max(g_cl - g_pl, 1e-6) * 1e-3
    return {"workload": "closure_98k_N3", "hexes": 6 * panel_n * panel_n * radial_n,
            "dof_updates_per_s": {k: c[k]["dof_updates_per_s"] for k in ("closure", "plain", "resolved")},
            "seconds_per_unit_time": {k: c[k]["seconds_per_time"] for k in ("closure", "plain", "resolved")},
            "cost_ratio_resolved_over_closure": c["ratio_resolved_over_closure"],
            "grad_kernel_ms": {"closure": g_cl, "plain": g_pl},
            "mlp": {"bound": "mfma", "achieved": flops / dt_mlp / 1e12, "peak": 2500.0, "unit": "TFLOP/s",
                    "frac": flops / dt_mlp / 1e12 / 2500.0, "alg_flops_per_launch": flops,
                    "note": "network time = the network pass plus the order-3 flux pass, minus the plain "
                            "order-3 flux pass"},
            "training": training_leg()}


def training_leg(iters=200):
    """Closure training (FP32 matrix-core products): Adam iterations on
    synthetic normalised samples, batch 4,096; about 3 x 12,672 flops per
    sample (forward, and a backward twice its size)."""
    import torch
    from chorus_inputs import mlp_init
    n, batch = 1 << 20, 4096
    gen = torch.Generator(device="cuda").manual_seed(0)
    X = torch.randn((n, 20), generator=gen, device="cuda", dtype=torch.float32)
    Y = torch.randn((n, 15), generator=gen, device="cuda", dtype=torch.float32)
    idx = torch.randint(0, n, (iters * batch,), generator=gen, device="cuda", dtype=torch.int32)
    P = torch.as_tensor(mlp_init(0), dtype=torch.float32).cuda()
    M, V = torch.zeros_like(P), torch.zeros_like(P)
    losses = torch.zeros(iters, dtype=torch.float32, device="cuda")
    from paper_1503_00834_amd import closure_train_workspace, chorus_closure_train
    ws = closure_train_workspace(batch)
    chorus_closure_train(X, Y, idx, batch, 10, P, M, V, 0, (1e-3, 0.9, 0.999, 1e-8), losses, ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    chorus_closure_train(X, Y, idx, batch, iters, P, M, V, 10, (1e-3, 0.9, 0.999, 1e-8), losses, ws)
    torch.cuda.synchronize()
    wt = time.perf_counter() - t0
    train_sps = iters * batch / wt
    del X, Y, idx, ws
    return {"samples_per_s": train_sps, "batch": batch, "iters": iters,
            "achieved": train_sps * 3 * 12672.0 / 1e12, "unit": "TFLOP/s (FP32 matrix)", "peak": 157.3}


def workload_leg(ch, workload, steps=20, repeats=3):
    """Both paths on another workload (DOF-updates/s: median of `repeats`
    timed calls of `steps` SSP-RK3 steps after two warm-up steps)."""
    import torch
    from chorus_inputs import CONFIGS, shell_params_from_config, uniform_noise
    cfg = CONFIGS[workload]
    ri, ro = shell_params_from_config(cfg)
    mesh = ch.chorus_mesh_create(cfg["panel_n"], cfg["radial_n"], cfg["order"], ri, ro).upload()
    Qh, pars = mesh.init_polytrope(cfg["beta"], cfg["n_rho"], poly_n=cfg["poly_n"],
                                   noise=uniform_noise(mesh.n_solpts, cfg["seed"]), amp=1e-4)
    Q0h, _ = mesh.init_polytrope(cfg["beta"], cfg["n_rho"], poly_n=cfg["poly_n"])
    out = {"workload": workload, "hexes": mesh.n_elems, "dofs": mesh.n_solpts, "steps": steps, "repeats": repeats}
    N = cfg["order"]
    for name, prec in (("mixed", ch.CHORUS_MIXED), ("fp64", ch.CHORUS_FP64)):
        phys = ch.physics(GM=pars["GM"], omega=cfg["omega"], nu=cfg["nu"], kappa=cfg["kappa"],
                          T_top=pars["chi_o"], precision=prec)
        dt = mesh.stable_dt(phys, Qh, cfg["cfl"])
        ws = mesh.workspace(phys)
        if prec == ch.CHORUS_MIXED:
            ch.chorus_set_background(mesh, phys, torch.from_numpy(Q0h).cuda(), ws)
        Q = torch.from_numpy(Qh).cuda()
        ch.chorus_rk_step(mesh, phys, Q, dt, 2, ws)
        torch.cuda.synchronize()
        walls = []
        for _ in range(repeats):
            t0 = time.perf_counter()
            ch.chorus_rk_step(mesh, phys, Q, dt, steps, ws)
            torch.cuda.synchronize()
            walls.append(time.perf_counter() - t0)
        wall = statistics.median(walls)
        if not bool(torch.isfinite(Q).all()):
            raise RuntimeError("%s state became non-finite" % workload)
        value = mesh.n_solpts * steps / wall
        out[name] = {"value": value, "ms_per_step": wall / steps * 1e3,
                     "path_hbm_frac": value * ALG_BYTES_PER_DOF_UPDATE[name][N] / (HBM_PEAK_GBS * 1e9)}
        del Q, ws
    return out


def next_rows_leg(ch, mesh, cfg, pars, Qh, Q0h, dt, ws, steps=10):
    """The rows built after the hot path, on the same workload and mixed
    path: the paper's five-stage fourth-order SSP integrator (DOF-updates/s,
    one update = one five-stage step), the solar radius-dependent radiative
    diffusivity (SSP-RK3 DOF-updates/s with the radial variant of the flux
    pass), and the angular-momentum correction (six fixed-order sums and the
    rigid-rotation removal, wall time per call including its host sync)."""
    import torch
    out = {}
    kw = dict(GM=pars["GM"], omega=cfg["omega"], nu=cfg["nu"], kappa=cfg["kappa"], T_top=pars["chi_o"],
              precision=ch.CHORUS_MIXED)

    def run(phys):
        ch.chorus_set_background(mesh, phys, torch.from_numpy(Q0h).cuda(), ws)
        Q = torch.from_numpy(Qh).cuda()
        ch.chorus_rk_step(mesh, phys, Q, dt, 1, ws)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ch.chorus_rk_step(mesh, phys, Q, dt, steps, ws)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        if not bool(torch.isfinite(Q).all()):
            raise RuntimeError("state became non-finite")
        return {"value": mesh.n_solpts * steps / wall, "ms_per_step": wall / steps * 1e3, "steps": steps}, Q

    r54, _ = run(ch.physics(integrator=ch.CHORUS_SSPRK54, **kw))
    out["ssprk54"] = dict(r54, unit="DOF-updates/s (five-stage steps)")
    k0, k1, k2 = ch.solar_radiative_diffusivity(cfg["beta"], cfg["n_rho"], 2e-3, poly_n=cfg["poly_n"])
    rkr, Q = run(ch.physics(kappa_r=k0, kappa_r1=k1, kappa_r2=k2, **kw))
    out["radial_kappa_r"] = dict(rkr, unit="DOF-updates/s", kappa_r=[k0, k1, k2])
    ch.chorus_am_correct(mesh, Q, ws)
    n = 20
    t0 = time.perf_counter()
    for _ in range(n):
        ch.chorus_am_correct(mesh, Q, ws)
    wall = (time.perf_counter() - t0) / n
    # per call and point: the sums read the coordinates, the weight, density
    # and momentum (8 doubles); the update reads the coordinates, density,
    # momentum and energy (8) and writes momentum and energy (4)
    nbytes = mesh.n_solpts * 8 * (8 + 8 + 4)
    out["am_correct"] = {"us_per_call": wall * 1e6, "hbm_GBs_incl_sync": nbytes / wall / 1e9}
    del Q
    return out


def size_sweep(ch):
    """DOF-updates/s of both paths (SSP-RK3) on cubed-sphere shells of the
    benchmark's stratification (beta 0.75, N_rho 3) from 288 to 331,776
    hexes at N = 4: where the GPU fills."""
    import torch
    rows = []
    for panel_n, radial_n in ((4, 3), (8, 4), (12, 6), (24, 12), (48, 24)):
        beta, n_rho = 0.75, 3.0
        ri, ro = beta / (1 - beta), 1 / (1 - beta)
        mesh = ch.chorus_mesh_create(panel_n, radial_n, 4, ri, ro).upload()
        Qh, pars = mesh.init_polytrope(beta, n_rho, noise=uniform_noise_of(mesh.n_solpts), amp=1e-4)
        Q0h, _ = mesh.init_polytrope(beta, n_rho)
        steps = max(5, min(200, int(4e7 / mesh.n_solpts)))
        row = {"hexes": mesh.n_elems, "dofs": mesh.n_solpts, "steps": steps}
        for name, prec in (("mixed", ch.CHORUS_MIXED), ("fp64", ch.CHORUS_FP64)):
            phys = ch.physics(GM=pars["GM"], omega=1.0, nu=2e-4, kappa=2e-4, T_top=pars["chi_o"], precision=prec)
            dt = mesh.stable_dt(phys, Qh, 0.5)
            ws = mesh.workspace(phys)
            if prec == ch.CHORUS_MIXED:
                ch.chorus_set_background(mesh, phys, torch.from_numpy(Q0h).cuda(), ws)
            Q = torch.from_numpy(Qh).cuda()
            ch.chorus_rk_step(mesh, phys, Q, dt, 2, ws)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ch.chorus_rk_step(mesh, phys, Q, dt, steps, ws)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            if not bool(torch.isfinite(Q).all()):
                raise RuntimeError("state became non-finite")
            row[name] = mesh.n_solpts * steps / wall
            del Q, ws
        log("size sweep: %s" % row)
        rows.append(row)
        del mesh
        torch.cuda.empty_cache()
    return rows


def uniform_noise_of(n):
    from chorus_inputs import uniform_noise
    return uniform_noise(n, 0)


def cpu_baseline(sample="jupiter_41k_N4", all_steps=2, single_steps=1):
    """The CPU oracle (FP64, plain C, OpenMP over elements) on a bounded
    sample of the workload: the 41,472-hex N = 4 shell, one eighth of the
    331,776-hex shell's elements (one GPU's share of it in an eight-way
    lateral split) with the same order and per-element work, timed on all
    the host cores of this process and on one thread.  The rate is per DOF,
    so it carries over to the full workload's unit."""
    import oracle
    from chorus_inputs import CONFIGS, cubed_sphere_shell, shell_params_from_config, uniform_noise
    oracle.build(force=False)
    cfg = CONFIGS[sample]
    ri, ro = shell_params_from_config(cfg)
    om = oracle.OracleMesh(cubed_sphere_shell(cfg["panel_n"], cfg["radial_n"], ri, ro), cfg["order"])
    Q, pars = om.polytrope(cfg["beta"], cfg["n_rho"], poly_n=cfg["poly_n"],
                           noise=uniform_noise(om.n_solpts, cfg["seed"]), amp=1e-4)
    ph = oracle.phys(GM=pars["GM"], omega=cfg["omega"], nu=cfg["nu"], kappa=cfg["kappa"],
                     T_top=pars["chi_o"])
    try:
        n_cpu = len(os.sched_getaffinity(0))
    except AttributeError:
        n_cpu = os.cpu_count() or 1
    threads_all = oracle.max_threads()

    def timed(threads, steps):
        oracle.set_threads(threads)
        t0 = time.perf_counter()
        om.rk3(ph, Q, 1e-3, steps)
        return om.n_solpts * steps / (time.perf_counter() - t0)

    v_all = timed(threads_all, all_steps)
    v_one = timed(1, single_steps)
    oracle.set_threads(threads_all)
    return {"value": v_all, "unit": "DOF-updates/s", "cores": threads_all, "kind": "oracle",
            "sample": "%d SSP-RK3 step(s) of the %d-hex N=%d shell (%s: 1/8 of the 331,776-hex "
                      "workload's elements, same order and per-element work), %d OpenMP threads"
                      % (all_steps, om.E, cfg["order"], sample, threads_all),
            "single_thread": {"value": v_one, "steps": single_steps, "cores": 1},
            "host_cpus": n_cpu}


def run_path(ch, mesh, phys, Q, dt, ws, args, stream, label):
    import torch
    log("%s: warm-up %d steps" % (label, args.warmup))
    ch.chorus_rk_step(mesh, phys, Q, dt, args.warmup, ws, stream)
    torch.cuda.synchronize()
    reps = []
    for r in range(args.repeats):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ch.chorus_rk_step(mesh, phys, Q, dt, args.steps, ws, stream)
        torch.cuda.synchronize()
        reps.append(time.perf_counter() - t0)
        log("%s: repeat %d: %.3f ms/step" % (label, r, reps[-1] / args.steps * 1e3))
    # the kernels' launch durations: one more K-step run with HIP events on
    # the launch stream (not part of the value)
    ch.chorus_kernel_timing(True)
    torch.cuda.synchronize()
    ch.chorus_rk_step(mesh, phys, Q, dt, args.steps, ws, stream)
    torch.cuda.synchronize()
    ch.chorus_kernel_timing(False)
    kt = ch.chorus_kernel_times()
    log("%s: kernel times %s" % (label, kt))
    return statistics.median(reps), reps, kt


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--repeats", type=int, default=5)
    ap.add_argument("--workload", default="sun_332k_N4")
    ap.add_argument("--precision", default="mixed", choices=["fp64", "mixed"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-closure", action="store_true", help="skip the learned-closure leg")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64-plain comparison on the same run")
    ap.add_argument("--no-other", action="store_true", help="skip the 41,472-hex workload leg")
    ap.add_argument("--no-next", action="store_true",
                    help="skip the leg of the five-stage integrator, radial kappa_r and angular-momentum correction")
    ap.add_argument("--closure-experiment", action="store_true",
                    help="only run the closure experiment at the configured sizes (about 5 minutes; one JSON line)")
    ap.add_argument("--closure-cost", action="store_true",
                    help="only time the resolved, plain and closure runs on the closure-run shell "
                         "(98,304 hexes; one JSON line; for profiling the order-3 passes)")
    ap.add_argument("--closure-training", type=int, default=0, metavar="ITERS",
                    help="only time this many closure training iterations (batch 4,096; one JSON line; for "
                         "profiling the training kernels)")
    ap.add_argument("--size-sweep", action="store_true",
                    help="only measure both paths on shells from 288 to 331,776 hexes (one JSON line)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MiB",
                    help="only run a plain device copy of this many MiB 5 times (HBM counter "
                         "calibration under rocprofv3 --pmc)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.steps < 1 or args.repeats < 1 or args.warmup < 0:
        print("need --steps >= 1, --repeats >= 1, --warmup >= 0", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1503_00834_amd as ch
    from chorus_inputs import CONFIGS, shell_params_from_config, uniform_noise

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    if args.copy_calibration:
        nbytes = args.copy_calibration << 20
        a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "launches": 5}))
        return
    if args.closure_experiment:
        from paper_1503_00834_amd import closure
        rep = closure.configured_experiment()
        print(json.dumps({"closure_experiment": rep, "data": "synthetic"}), flush=True)
        return
    if args.closure_cost:
        from paper_1503_00834_amd import closure
        c = closure.cost_per_time(32, 16, steps=1)
        print(json.dumps({"closure_cost": c, "data": "synthetic"}), flush=True)
        return
    if args.closure_training:
        print(json.dumps({"closure_training": training_leg(args.closure_training), "data": "synthetic"}),
              flush=True)
        return
    if args.size_sweep:
        print(json.dumps({"size_sweep": size_sweep(ch), "unit": "DOF-updates/s", "integrator": "SSP-RK3",
                          "order": 4, "data": "synthetic"}), flush=True)
        return
    cfg = CONFIGS[args.workload]
    N = cfg["order"]
    ri, ro = shell_params_from_config(cfg)
    log("workload %s: building mesh" % args.workload)
    mesh = ch.chorus_mesh_create(cfg["panel_n"], cfg["radial_n"], N, ri, ro).upload()
    noise = uniform_noise(mesh.n_solpts, cfg["seed"])
    Qh, pars = mesh.init_polytrope(cfg["beta"], cfg["n_rho"], poly_n=cfg["poly_n"], noise=noise, amp=1e-4)
    del noise
    prec = ch.CHORUS_MIXED if args.precision == "mixed" else ch.CHORUS_FP64
    kw = dict(GM=pars["GM"], omega=cfg["omega"], nu=cfg["nu"], kappa=cfg["kappa"], T_top=pars["chi_o"])
    phys = ch.physics(precision=prec, **kw)
    dt = mesh.stable_dt(phys, Qh, cfg["cfl"])
    Q = torch.from_numpy(Qh).cuda()
    ws = mesh.workspace(phys)
    Q0h = None
    if prec == ch.CHORUS_MIXED:
        # background: the polytrope without the perturbation (at rest)
        Q0h, _ = mesh.init_polytrope(cfg["beta"], cfg["n_rho"], poly_n=cfg["poly_n"])
        ch.chorus_set_background(mesh, phys, torch.from_numpy(Q0h).cuda(), ws)
    log("E=%d N=%d DOFs=%d dt=%.3e; warmup %d, %d x %d timed steps" % (
        mesh.n_elems, N, mesh.n_solpts, dt, args.warmup, args.repeats, args.steps))
    stream = torch.cuda.current_stream()
    med, reps, ktimes = run_path(ch, mesh, phys, Q, dt, ws, args, stream, args.precision)
    total_steps = args.warmup + (args.repeats + 1) * args.steps

    # sanity outside the timed region
    if not bool(torch.isfinite(Q).all()) or not bool((Q[0] > 0).all()):
        print("state became non-finite or non-positive", file=sys.stderr)
        sys.exit(3)

    value = mesh.n_solpts * args.steps / med
    # dominant kernel: the pass with the longer average launch (the flux pass
    # of either path); it carries the line operators and pointwise fluxes, so
    # the stage's algorithmic bytes (and flops) are set against its launch time
    per_launch = {k: ktimes[k][0] / max(ktimes[k][1], 1) for k in ("pass1", "pass2")}
    dom = max(per_launch, key=per_launch.get)
    kname = ch.KERNEL_NAMES[args.precision][dom]
    avg_s = per_launch[dom] * 1e-3
    alg = alg_bytes_per_stage_point(N, args.precision) * mesh.n_solpts
    achieved = alg / avg_s / 1e9
    flops = alg_flops_per_stage_point(N) * mesh.n_solpts
    tflops = flops / avg_s / 1e12
    peak_alu = ALU_PEAK_TFLOPS[args.precision]
    path_gbs = value * ALG_BYTES_PER_DOF_UPDATE[args.precision][N] / 1e9
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "DOF-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": med / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "hexes": mesh.n_elems, "order": N, "dofs": mesh.n_solpts,
                   "precision": args.precision, "integrator": "SSP-RK3", "dt": dt,
                   "repeats": args.repeats, "timing": "median of the repeats, per-kernel events off"},
        "repeats_ms_per_step": [r / args.steps * 1e3 for r in reps],
        "roofline": {"bound": "hbm", "kernel": kname, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(args.workload, args.precision, kname),
                     "alg_bytes_per_launch": alg, "avg_launch_ms": avg_s * 1e3,
                     "alg_bytes_per_dof_update": ALG_BYTES_PER_DOF_UPDATE[args.precision][N],
                     "path": {"achieved": path_gbs, "unit": "GB/s", "frac": path_gbs / HBM_PEAK_GBS,
                              "note": "whole SSP-RK3 step: DOF-updates/s x algorithmic bytes per DOF-update"},
                     "alu": {"achieved": tflops, "peak": peak_alu, "unit": "TFLOP/s", "frac": tflops / peak_alu,
                             "alg_flops_per_launch": flops}},
        "kernels_ms_per_step": {ch.KERNEL_NAMES[args.precision][k]: v[0] / args.steps for k, v in ktimes.items()},
        "kernels_avg_launch_ms": {ch.KERNEL_NAMES[args.precision][k]: v[0] / max(v[1], 1)
                                  for k, v in ktimes.items()},
    }
    if prec == ch.CHORUS_MIXED and not args.no_fp64:
        # the FP64 plain path on the same workload, for the comparison the
        # metric names: the same warm-up and timed steps from the same state,
        # so the two end states can be compared (outside the timing)
        log("fp64 plain path on the same run")
        p64 = ch.physics(precision=ch.CHORUS_FP64, **kw)
        Q64 = torch.from_numpy(Qh).cuda()
        med64, reps64, kt64 = run_path(ch, mesh, p64, Q64, dt, ws, args, stream, "fp64")
        Qs = torch.from_numpy(Qh).cuda()
        rel, rel_change = [], []
        for v in range(5):
            d = torch.linalg.vector_norm(Q[v] - Q64[v]).item()
            rel.append(d / torch.linalg.vector_norm(Q64[v]).item())
            rel_change.append(d / max(torch.linalg.vector_norm(Q64[v] - Qs[v]).item(), 1e-300))
        del Qs
        v64 = mesh.n_solpts * args.steps / med64
        out["fp64_plain"] = {"value": v64, "ms_per_step": med64 / args.steps * 1e3,
                             "repeats_ms_per_step": [r / args.steps * 1e3 for r in reps64],
                             "speedup_mixed_over_fp64": med64 / med,
                             "kernels_avg_launch_ms": {ch.KERNEL_NAMES["fp64"][k]: t[0] / max(t[1], 1)
                                                       for k, t in kt64.items()},
                             "path_hbm_frac": v64 * ALG_BYTES_PER_DOF_UPDATE["fp64"][N] / (HBM_PEAK_GBS * 1e9),
                             "mixed_vs_fp64": {"steps": total_steps, "rel_l2_per_variable": rel,
                                               "max_rel_l2": max(rel), "bound": 1e-6,
                                               "rel_to_change_per_variable": rel_change}}
        log("mixed vs fp64 after %d steps: %s" % (total_steps, rel))
        del Q64
    if prec == ch.CHORUS_MIXED and not args.no_next:
        log("five-stage integrator, radial kappa_r, angular-momentum leg")
        out["next_rows"] = next_rows_leg(ch, mesh, cfg, pars, Qh, Q0h, dt, ws)
        torch.cuda.synchronize()
    del Q, ws
    torch.cuda.empty_cache()
    if not args.no_other:
        other = "jupiter_41k_N4" if args.workload != "jupiter_41k_N4" else "sun_332k_N4"
        log("%s leg" % other)
        out["other_workload"] = workload_leg(ch, other)
        torch.cuda.synchronize()
    if not args.no_closure:
        log("closure leg")
        out["closure"] = closure_leg()
        torch.cuda.synchronize()
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
