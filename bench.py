#!/usr/bin/env python3
"""Benchmark: SD DOF-updates/s of the SSP-RK3 spectral-difference solver on
one MI355X, with the per-kernel HBM roofline and the CPU oracle beside it.

One step = one full SSP-RK3 step (three residual evaluations with the fused
stage update) over every solution point of the workload; DOFs = E N^3.
Inputs are synthetic and seeded: a cubed-sphere shell, the polytropic
background and a seeded entropy perturbation (see the design notes).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

Prints one JSON line.
"""
import argparse
import json
import os
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


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def alg_bytes_per_stage_point(N, precision):
    """Algorithmic bytes per solution point and residual stage.

    FP64 state: 5 reads + 3 writes of 40 B per point per SSP-RK3 step, i.e.
    320/3 B per stage; geometry from the 20 element nodes (480 B) and the
    face connectivity (48 B) once per element and stage."""
    NP = N ** 3
    per = 320.0 / 3.0 + (480.0 + 48.0) / NP
    if precision == "mixed":
        # FP32 background residual (20 B), rho0, p0 (8 B) per point, and the
        # FP32 background face jump + wave speed (12 B per face point)
        per += 28.0 + 12.0 * 6 * N * N / NP
    return per


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
    import torch
    from paper_1503_00834_amd import closure
    from chorus_inputs import mlp_init
    c = closure.cost_per_time(panel_n, radial_n, kernel_times=True)
    # training (FP32, one thread per sample): Adam iterations on synthetic
    # normalised samples, batch 4,096; about 3 x 12,672 flops per sample
    # (forward, and a backward twice its size)
    n, batch, iters = 1 << 20, 4096, 200
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
            "training": {"samples_per_s": train_sps, "batch": batch, "iters": iters,
                         "achieved": train_sps * 3 * 12672.0 / 1e12, "unit": "TFLOP/s (FP32 vector)",
                         "peak": 157.3}}


def large_leg(ch, workload="sun_332k_N4", steps=10):
    """The mixed path on the largest shell (6 x 48 x 48 x 24 = 331,776 hexes,
    N = 4, 21.2M DOFs, 849 MB per FP64 state copy), which no cache holds:
    DOF-updates/s over a few SSP-RK3 steps after one warm-up step."""
    import torch
    from chorus_inputs import CONFIGS, shell_params_from_config, uniform_noise
    cfg = CONFIGS[workload]
    ri, ro = shell_params_from_config(cfg)
    mesh = ch.chorus_mesh_create(cfg["panel_n"], cfg["radial_n"], cfg["order"], ri, ro).upload()
    Qh, pars = mesh.init_polytrope(cfg["beta"], cfg["n_rho"], poly_n=cfg["poly_n"],
                                   noise=uniform_noise(mesh.n_solpts, cfg["seed"]), amp=1e-4)
    phys = ch.physics(GM=pars["GM"], omega=cfg["omega"], nu=cfg["nu"], kappa=cfg["kappa"],
                      T_top=pars["chi_o"], precision=ch.CHORUS_MIXED)
    dt = mesh.stable_dt(phys, Qh, cfg["cfl"])
    ws = mesh.workspace(phys)
    Q0h, _ = mesh.init_polytrope(cfg["beta"], cfg["n_rho"], poly_n=cfg["poly_n"])
    ch.chorus_set_background(mesh, phys, torch.from_numpy(Q0h).cuda(), ws)
    del Q0h
    Q = torch.from_numpy(Qh).cuda()
    stream = torch.cuda.current_stream()
    ch.chorus_rk_step(mesh, phys, Q, dt, 1, ws, stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ch.chorus_rk_step(mesh, phys, Q, dt, steps, ws, stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    if not bool(torch.isfinite(Q).all()):
        raise RuntimeError("large workload state became non-finite")
    value = mesh.n_solpts * steps / wall
    N = cfg["order"]
    return {"workload": workload, "hexes": mesh.n_elems, "dofs": mesh.n_solpts, "precision": "mixed",
            "steps": steps, "value": value, "ms_per_step": wall / steps * 1e3,
            "path_hbm_frac": value * alg_bytes_per_stage_point(N, "mixed") * 3.0 / (HBM_PEAK_GBS * 1e9)}


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


def cpu_baseline(cfg, budget_s=15.0):
    """The CPU oracle on the same workload for a bounded number of steps."""
    import oracle
    from chorus_inputs import cubed_sphere_shell, shell_params_from_config, uniform_noise
    oracle.build(force=False)
    ri, ro = shell_params_from_config(cfg)
    m = cubed_sphere_shell(cfg["panel_n"], cfg["radial_n"], ri, ro)
    om = oracle.OracleMesh(m, cfg["order"])
    Q, pars = om.polytrope(cfg["beta"], cfg["n_rho"], poly_n=cfg["poly_n"],
                           noise=uniform_noise(om.n_solpts, cfg["seed"]), amp=1e-4)
    ph = oracle.phys(GM=pars["GM"], omega=cfg["omega"], nu=cfg["nu"], kappa=cfg["kappa"],
                     T_top=pars["chi_o"])
    dt = 1e-3
    steps, t0 = 0, time.perf_counter()
    while True:
        Q = om.rk3(ph, Q, dt, 1)
        steps += 1
        el = time.perf_counter() - t0
        if el >= budget_s or steps >= 20:
            break
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": om.n_solpts * steps / el, "unit": "DOF-updates/s", "cores": threads,
            "kind": "oracle",
            "sample": "%d SSP-RK3 step(s) of the full workload (%d hexes, N=%d), %.1f s" % (
                steps, om.E, cfg["order"], el)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="jupiter_41k_N4")
    ap.add_argument("--precision", default="mixed", choices=["fp64", "mixed"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-closure", action="store_true", help="skip the learned-closure leg")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64-plain comparison leg")
    ap.add_argument("--no-large", action="store_true", help="skip the 331,776-hex shell leg")
    ap.add_argument("--no-next", action="store_true",
                    help="skip the leg of the five-stage integrator, radial kappa_r and angular-momentum correction")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--size-sweep", action="store_true",
                    help="only measure both paths on shells from 288 to 331,776 hexes (one JSON line)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MiB",
                    help="only run a plain device copy of this many MiB 5 times (HBM counter "
                         "calibration under rocprofv3 --pmc)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
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
    prec = ch.CHORUS_MIXED if args.precision == "mixed" else ch.CHORUS_FP64
    phys = ch.physics(GM=pars["GM"], omega=cfg["omega"], nu=cfg["nu"], kappa=cfg["kappa"],
                      T_top=pars["chi_o"], precision=prec)
    dt = mesh.stable_dt(phys, Qh, cfg["cfl"])
    Q = torch.from_numpy(Qh).cuda()
    ws = mesh.workspace(phys)
    if prec == ch.CHORUS_MIXED:
        # background: the polytrope without the perturbation (at rest)
        Q0h, _ = mesh.init_polytrope(cfg["beta"], cfg["n_rho"], poly_n=cfg["poly_n"])
        ch.chorus_set_background(mesh, phys, torch.from_numpy(Q0h).cuda(), ws)
    log("E=%d N=%d DOFs=%d dt=%.3e; warmup %d" % (mesh.n_elems, N, mesh.n_solpts, dt, args.warmup))
    stream = torch.cuda.current_stream()
    ch.chorus_rk_step(mesh, phys, Q, dt, args.warmup, ws, stream)
    torch.cuda.synchronize()

    log("timing %d steps" % args.steps)
    ch.chorus_kernel_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ch.chorus_rk_step(mesh, phys, Q, dt, args.steps, ws, stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ch.chorus_kernel_timing(False)
    ktimes = ch.chorus_kernel_times()
    log("kernel times: %s" % ktimes)

    # sanity outside the timed region
    Qc = Q.cpu().numpy()
    if not np.isfinite(Qc).all() or (Qc[0] <= 0).any():
        print("state became non-finite or non-positive", file=sys.stderr)
        sys.exit(3)

    dof_updates = mesh.n_solpts * args.steps
    value = dof_updates / wall
    # dominant kernel: the pass with the longer average launch (the flux pass
    # of either path); it carries the line operators and pointwise fluxes, so
    # the stage's algorithmic flops and bytes are set against its launch time
    per_launch = {k: ktimes[k][0] / max(ktimes[k][1], 1) for k in ("pass1", "pass2")}
    dom = max(per_launch, key=per_launch.get)
    kname = ch.KERNEL_NAMES[args.precision][dom]
    avg_s = per_launch[dom] * 1e-3
    alg = alg_bytes_per_stage_point(N, args.precision) * mesh.n_solpts
    achieved = alg / avg_s / 1e9
    flops = alg_flops_per_stage_point(N) * mesh.n_solpts
    tflops = flops / avg_s / 1e12
    peak_alu = ALU_PEAK_TFLOPS[args.precision]
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "DOF-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "hexes": mesh.n_elems, "order": N, "dofs": mesh.n_solpts,
                   "precision": args.precision, "integrator": "SSP-RK3", "dt": dt},
        "roofline": {"bound": "alu", "kernel": kname, "achieved": tflops, "peak": peak_alu,
                     "unit": "TFLOP/s", "frac": tflops / peak_alu,
                     "traffic": measured_traffic(args.workload, args.precision, kname),
                     "alg_flops_per_launch": flops, "avg_launch_ms": avg_s * 1e3,
                     "hbm": {"achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                             "frac": achieved / HBM_PEAK_GBS, "alg_bytes_per_launch": alg},
                     "path_hbm_frac": value * alg_bytes_per_stage_point(N, args.precision) * 3.0
                     / (HBM_PEAK_GBS * 1e9)},
        "kernels_ms_per_step": {ch.KERNEL_NAMES[args.precision][k]: v[0] / args.steps for k, v in ktimes.items()},
    }
    if prec == ch.CHORUS_MIXED and not args.no_fp64:
        # the FP64 plain path on the same workload, for the comparison the
        # metric names: the same untimed and timed steps from the same
        # state, so the two end states can be compared (outside the timing)
        log("fp64 plain path")
        p64 = ch.physics(GM=pars["GM"], omega=cfg["omega"], nu=cfg["nu"], kappa=cfg["kappa"],
                         T_top=pars["chi_o"], precision=ch.CHORUS_FP64)
        Q64 = torch.from_numpy(Qh).cuda()
        ch.chorus_rk_step(mesh, p64, Q64, dt, args.warmup, ws, stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ch.chorus_rk_step(mesh, p64, Q64, dt, args.steps, ws, stream)
        torch.cuda.synchronize()
        w64 = time.perf_counter() - t0
        A = Q64.cpu().numpy().reshape(5, -1)
        B = Qc.reshape(5, -1)
        start = Qh.reshape(5, -1)
        rel = [float(np.linalg.norm(B[v] - A[v]) / np.linalg.norm(A[v])) for v in range(5)]
        rel_change = [float(np.linalg.norm(B[v] - A[v]) / max(np.linalg.norm(A[v] - start[v]), 1e-300))
                      for v in (0, 4)]
        out["fp64_plain"] = {"value": mesh.n_solpts * args.steps / w64, "ms_per_step": w64 / args.steps * 1e3,
                             "speedup_mixed_over_fp64": w64 / wall,
                             "mixed_vs_fp64": {"steps": args.warmup + args.steps, "rel_l2_per_variable": rel,
                                               "max_rel_l2": max(rel), "bound": 1e-6,
                                               "rel_to_change_rho_E": rel_change}}
        del Q64
    if prec == ch.CHORUS_MIXED and not args.no_next:
        log("five-stage integrator, radial kappa_r, angular-momentum leg")
        out["next_rows"] = next_rows_leg(ch, mesh, cfg, pars, Qh, Q0h, dt, ws)
        torch.cuda.synchronize()
    if prec == ch.CHORUS_MIXED and not args.no_large:
        log("large-shell leg")
        del Q, ws
        torch.cuda.empty_cache()
        out["large"] = large_leg(ch)
        torch.cuda.synchronize()
    if not args.no_closure:
        log("closure leg")
        out["closure"] = closure_leg()
        torch.cuda.synchronize()
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(cfg, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
