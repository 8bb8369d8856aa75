"""Learned subgrid closure: training data from resolved runs, training, and
the judge that keeps the closure only when it improves the coarse solve.

Host orchestration of library calls (every numerical step of the solver,
the filter, the features, training and inference runs in the library's HIP
kernels); PyTorch provides device memory, the normalisation statistics and
the judge's diagnostics.

Pipeline (the paper names subgrid modelling for large-eddy runs as the
code's next step, Summary; its diagnostics are the kinetic energy and mean
radial profiles of Section 7.2 and the velocity spectra of the benchmarks):

  1. resolved run at order N_f on a hex mesh (snapshots of Q);
  2. each snapshot filtered to order N_c on the same mesh
     (chorus_closure_filter): filtered state Qbar and subgrid flux
     tau = G F(Q) - F(G Q);
  3. features (Q, grad Q) of Qbar by the order-N_c solver's own BR1
     gradients (chorus_closure_features) -> samples X, targets Y = tau;
  4. normalisation from the training samples, mini-batch Adam
     (chorus_closure_train), packing (chorus_closure_pack);
  5. judge: coarse runs with and without the closure against the filtered
     resolved run at equal physical time, compared by the kinetic-energy
     spectrum and the mean radial profiles; the closure is kept only if it
     is finite and does not make these errors larger.
"""
import math

import numpy as np

from . import (CHORUS_CLOSURE_MLP, CHORUS_MLP_NPARAM, ChorusError, chorus_closure_features,
               chorus_closure_filter, chorus_closure_pack, chorus_closure_train, chorus_rk_step,
               closure_train_workspace, physics)


def _torch():
    import torch
    return torch


# ---------------------------------------------------------------------------
# data
# ---------------------------------------------------------------------------
def resolved_snapshots(mesh_f, phys_f, Q, dt, n_spinup, n_snap, every, ws=None):
    """Advance Q (device, order N_f) n_spinup steps, then record n_snap
    snapshots `every` steps apart (the first right after the spin-up).
    Returns (list of device copies, their times)."""
    ws = ws if ws is not None else mesh_f.workspace(phys_f)
    chorus_rk_step(mesh_f, phys_f, Q, dt, n_spinup, ws)
    snaps, times = [], []
    t = n_spinup * dt
    for i in range(n_snap):
        if i:
            chorus_rk_step(mesh_f, phys_f, Q, dt, every, ws)
            t += every * dt
        snaps.append(Q.clone())
        times.append(t)
    return snaps, times


def filter_to_coarse(mesh_f, mesh_c, gamma, Qf):
    """(Qbar [5, E Nc^3], tau [15, E Nc^3]) float64 device tensors."""
    torch = _torch()
    Qb = torch.empty((5, mesh_c.n_solpts), dtype=torch.float64, device=Qf.device)
    tau = torch.empty((15, mesh_c.n_solpts), dtype=torch.float64, device=Qf.device)
    chorus_closure_filter(mesh_f, mesh_c, gamma, Qf, Qb, tau)
    return Qb, tau


def samples(mesh_f, mesh_c, phys_c, snapshots, gamma, ws_c=None):
    """Raw features X [n, 20] and targets Y [n, 15] (float32, device) from
    the filtered snapshots."""
    torch = _torch()
    ws_c = ws_c if ws_c is not None else mesh_c.workspace(phys_c)
    Xs, Ys = [], []
    for Qf in snapshots:
        Qb, tau = filter_to_coarse(mesh_f, mesh_c, gamma, Qf)
        X = torch.empty((mesh_c.n_solpts, 20), dtype=torch.float32, device=Qf.device)
        chorus_closure_features(mesh_c, phys_c, Qb, X, ws_c)
        Xs.append(X)
        Ys.append(tau.t().to(torch.float32).contiguous())
    return torch.cat(Xs), torch.cat(Ys)


def normalisation(X, Y, eps=1e-30):
    """x_mean, x_inv_std, y_mean, y_std (70 floats, device) from the
    training samples; outputs with zero spread (the mass flux) get
    y_std = 0, i.e. the network never produces them."""
    torch = _torch()
    X64, Y64 = X.to(torch.float64), Y.to(torch.float64)
    xm, xs = X64.mean(0), X64.std(0)
    ym, ys = Y64.mean(0), Y64.std(0)
    xinv = torch.where(xs > eps, 1.0 / xs.clamp_min(eps), torch.zeros_like(xs))
    ys = torch.where(ys > eps, ys, torch.zeros_like(ys))
    ym = torch.where(ys > 0, ym, torch.zeros_like(ym))
    return torch.cat([xm, xinv, ym, ys]).to(torch.float32).contiguous()


def normalised(X, Y, norm):
    torch = _torch()
    n = norm.to(torch.float64)
    Xn = ((X.to(torch.float64) - n[0:20]) * n[20:40]).to(torch.float32).contiguous()
    ys = n[55:70]
    Yn = torch.where(ys > 0, (Y.to(torch.float64) - n[40:55]) / torch.where(ys > 0, ys, torch.ones_like(ys)),
                     torch.zeros_like(Y, dtype=torch.float64))
    return Xn, Yn.to(torch.float32).contiguous()


def train(X, Y, norm, params0, iters, batch, seed, lr=1e-3, betas=(0.9, 0.999), eps=1e-8, chunk=500):
    """Mini-batch Adam on the normalised samples; the sample order is a
    seeded sequence of permutations (numpy PCG64), passed to the kernels.
    Returns (params, per-iteration losses)."""
    torch = _torch()
    Xn, Yn = normalised(X, Y, norm)
    n = Xn.shape[0]
    rng = np.random.Generator(np.random.PCG64(int(seed)))
    need = iters * batch
    order = np.concatenate([rng.permutation(n) for _ in range(need // n + 1)])[:need].astype(np.int32)
    idx = torch.from_numpy(order).to(X.device)
    P = torch.as_tensor(params0, dtype=torch.float32).to(X.device).contiguous()
    assert P.numel() == CHORUS_MLP_NPARAM
    M, V = torch.zeros_like(P), torch.zeros_like(P)
    losses = torch.zeros(iters, dtype=torch.float32, device=X.device)
    ws = closure_train_workspace(batch, device=X.device)
    done = 0
    while done < iters:
        k = min(chunk, iters - done)
        chorus_closure_train(Xn, Yn, idx[done * batch:], batch, k, P, M, V, done, (lr, betas[0], betas[1], eps),
                             losses[done:], ws)
        done += k
    return P, losses


def apriori_r2(mesh_c, phys_cl, Qbar, tau, ws=None):
    """Per-output fraction of the target variance explained by the packed
    network, evaluated by the fused bfloat16 inference on the filtered
    state Qbar against the filtered targets tau [15, n]."""
    from . import chorus_closure_infer
    torch = _torch()
    ws = ws if ws is not None else mesh_c.workspace(phys_cl)
    sgs = torch.empty((15, mesh_c.n_solpts), dtype=torch.float32, device=Qbar.device)
    chorus_closure_infer(mesh_c, phys_cl, Qbar, sgs, ws)
    T = tau.double()
    var = ((T - T.mean(1, keepdim=True)) ** 2).sum(1)
    res = ((T - sgs.double()) ** 2).sum(1)
    r2 = torch.where(var > 0, 1.0 - res / torch.where(var > 0, var, torch.ones_like(var)),
                     torch.full_like(var, float("nan")))
    return r2.cpu().numpy(), sgs


# ---------------------------------------------------------------------------
# judge (diagnostics of Section 7.2 and the benchmarks' spectra)
# ---------------------------------------------------------------------------
class ShellDiagnostics:
    """Radial bins and spherical-harmonic basis on the solution points of a
    shell mesh (host arrays)."""

    def __init__(self, mesh, r_inner, r_outer, n_bins=None, l_max=10, top_depth=None):
        """top_depth: thickness of the outer layer whose velocity is
        projected on the spherical harmonics; it should cover whole element
        layers (all solution points of a radial column), which makes the
        solution-point quadrature of the projection accurate (default: the
        whole shell)."""
        xyz, wJ = mesh.solpts()
        self.w = wJ
        r = np.sqrt((xyz ** 2).sum(0))
        self.r = r
        nb = n_bins or 2 * mesh.order
        edges = np.linspace(r_inner, r_outer, nb + 1)
        self.bin = np.clip(np.searchsorted(edges, r) - 1, 0, nb - 1)
        self.n_bins = nb
        self.r_mid = 0.5 * (edges[1:] + edges[:-1])
        self.bw = np.bincount(self.bin, weights=wJ, minlength=nb)
        # spectrum: volume-weighted projection of the top layer onto Y_lm
        depth = (r_outer - r_inner) if top_depth is None else top_depth
        top = r >= r_outer - depth * (1.0 + 1e-9)
        self.top = np.nonzero(top)[0]
        th = np.arccos(np.clip(xyz[2, self.top] / r[self.top], -1, 1))
        ph = np.arctan2(xyz[1, self.top], xyz[0, self.top])
        self.l_max = l_max
        self.Y = self._real_sh(l_max, th, ph)          # [(l, m) index][points]
        self.wt = wJ[self.top] / r[self.top] ** 2       # solid-angle weight of the layer

    @staticmethod
    def _real_sh(lmax, th, ph):
        """Real orthonormal spherical harmonics via associated Legendre
        functions (scipy), stacked for l <= lmax."""
        from scipy.special import lpmv
        rows, ls = [], []
        x = np.cos(th)
        for l in range(lmax + 1):
            for m in range(0, l + 1):
                norm = math.sqrt((2 * l + 1) / (4 * math.pi) * math.factorial(l - m) / math.factorial(l + m))
                P = lpmv(m, l, x) * norm * (-1) ** m
                if m == 0:
                    rows.append(P)
                    ls.append(l)
                else:
                    rows.append(math.sqrt(2) * P * np.cos(m * ph))
                    rows.append(math.sqrt(2) * P * np.sin(m * ph))
                    ls += [l, l]
        return np.array(rows), np.array(ls)

    def profiles(self, Q, gamma=5.0 / 3.0, R_gas=1.0):
        """Horizontal means per radial bin: rho, T, S, KE density, V_rms."""
        Q = Q.reshape(5, -1)
        rho, m, E = Q[0], Q[1:4], Q[4]
        ke = 0.5 * (m ** 2).sum(0) / rho
        p = (gamma - 1.0) * (E - ke)
        T = p / (rho * R_gas)
        cp = gamma * R_gas / (gamma - 1.0)
        S = cp * np.log(p ** (1.0 / gamma) / rho)
        v2 = (m ** 2).sum(0) / rho ** 2

        def hm(f):
            return np.bincount(self.bin, weights=f * self.w, minlength=self.n_bins) / self.bw
        return {"rho": hm(rho), "T": hm(T), "S": hm(S), "KE": hm(ke), "Vrms": np.sqrt(hm(v2))}

    def spectrum(self, Q):
        """E(l) = sum_m sum_c |<u_c, Y_lm>|^2 over the top layer."""
        Q = Q.reshape(5, -1)
        u = Q[1:4, self.top] / Q[0, self.top]
        Yv, ls = self.Y
        coef = (u[:, None, :] * Yv[None, :, :] * self.wt[None, None, :]).sum(-1) / self.wt.sum() * 4 * math.pi
        e = (coef ** 2).sum(0)
        return np.bincount(ls, weights=e, minlength=self.l_max + 1)


def judge_errors(diag, Q, Q_ref, gamma=5.0 / 3.0):
    """Relative errors of the KE spectrum (l >= 1) and of the mean profiles
    (rho, T, S, KE, V_rms; max over profiles) against a reference state."""
    s, s0 = diag.spectrum(Q), diag.spectrum(Q_ref)
    spec = float(np.linalg.norm(s[1:] - s0[1:]) / np.linalg.norm(s0[1:]))
    pr, pr0 = diag.profiles(Q, gamma), diag.profiles(Q_ref, gamma)
    prof = {}
    cp = gamma / (gamma - 1.0)
    for k in pr:
        a, b = pr[k], pr0[k]
        if k == "S":  # entropy is defined up to a constant: relative to c_p
            prof[k] = float(np.linalg.norm(a - b) / (cp * math.sqrt(len(b))))
        else:
            prof[k] = float(np.linalg.norm(a - b) / np.linalg.norm(b))
    return {"spectrum": spec, "profiles": prof, "profile_max": max(prof.values())}


def score(err):
    """Worst relative error over the judged statistics (KE spectrum and the
    mean profiles)."""
    return max(err["spectrum"], err["profile_max"])


def mean_errors(errs):
    """Time average of judge_errors() dictionaries."""
    keys = errs[0]["profiles"].keys()
    prof = {k: float(np.mean([e["profiles"][k] for e in errs])) for k in keys}
    return {"spectrum": float(np.mean([e["spectrum"] for e in errs])), "profiles": prof,
            "profile_max": max(prof.values())}


def choose(err_closure, err_plain, closure_finite=True):
    """Keep the closure only if its run stayed finite and its worst judged
    statistic is not worse than the plain run's."""
    if not closure_finite or err_closure is None:
        return False
    return score(err_closure) <= score(err_plain)


def judged_runs(mesh_c, diag, phys_plain, phys_closure, Q_start, refs, dt, steps_between, gamma=5.0 / 3.0):
    """Coarse runs with and without the closure from Q_start, compared with
    each reference state refs[i] (the filtered resolved run) after
    (i + 1) * steps_between steps.  Returns time-averaged errors per run
    (None for a run that became non-finite)."""
    torch = _torch()
    out = {}
    for name, ph in (("plain", phys_plain), ("closure", phys_closure)):
        if ph is None:
            out[name] = None
            continue
        ws = mesh_c.workspace(ph)
        q = Q_start.clone()
        errs = []
        for ref in refs:
            chorus_rk_step(mesh_c, ph, q, dt, steps_between, ws)
            if not bool(torch.isfinite(q).all()):
                errs = None
                break
            errs.append(judge_errors(diag, q.cpu().numpy(), ref.cpu().numpy(), gamma))
        out[name] = mean_errors(errs) if errs else None
    return out


def rejudge(report, params, norm):
    """Judge another parameter vector on the same runs as experiment()."""
    c = report["context"]
    model = pack_or_none(params, norm)
    if model is None:
        return False, None
    pcl = closure_physics(c["phys_kwargs"], model)
    errs = judged_runs(c["mesh"], c["diag"], physics(**c["phys_kwargs"]), pcl, c["start"], c["refs"], c["dt"],
                       c["steps"], c["phys_kwargs"]["gamma"])
    return choose(errs["closure"], errs["plain"], closure_finite=errs["closure"] is not None), errs


def pack_or_none(params, norm):
    """Packed model, or None when the parameters are unusable (NaN/Inf):
    the caller then runs the plain solve."""
    try:
        return chorus_closure_pack(params, norm)
    except ChorusError as e:
        if e.status == -5:
            return None
        raise


def closure_physics(base_kwargs, model):
    """physics() with the closure on (model not None) or off."""
    if model is None:
        return physics(**base_kwargs)
    return physics(closure=CHORUS_CLOSURE_MLP, closure_model=model, **base_kwargs)


def experiment(panel_n=6, radial_n=3, beta=0.7, n_rho=1.0, omega=0.5, nu=1e-3, vel_amp=0.15, k_range=(2.0, 6.0),
               order_fine=6, order_coarse=3, cfl=0.3, n_spinup=100, n_snap=60, n_train=30, every=20,
               iters=3000, batch=2048, lr=1e-3, seed=0, params0=None, gamma=5.0 / 3.0):
    """The whole closure pipeline on a seeded synthetic shell flow.

    Resolved run at order_fine from a polytrope (Section 4.2) carrying a
    seeded smooth random velocity field; snapshots 0..n_train-1 train the
    network, the rest are the reference for the judged coarse runs started
    from the filtered snapshot n_train (time step 2 dt_fine, so both reach
    the reference times).  Returns a report dict; report["model"] is the
    packed network (None if the parameters were non-finite) and
    report["use_closure"] the judge's decision."""
    import time
    from chorus_inputs import random_velocity, uniform_noise, mlp_init
    from . import chorus_mesh_create
    torch = _torch()
    ri, ro = beta / (1.0 - beta), 1.0 / (1.0 - beta)
    mf = chorus_mesh_create(panel_n, radial_n, order_fine, ri, ro).upload()
    mc = chorus_mesh_create(panel_n, radial_n, order_coarse, ri, ro).upload()
    Qh, pars = mf.init_polytrope(beta, n_rho, gamma=gamma, noise=uniform_noise(mf.n_solpts, seed), amp=1e-3)
    xyz, _ = mf.solpts()
    u = random_velocity(xyz, seed + 1, amp=vel_amp, k_min=k_range[0], k_max=k_range[1])
    Qh[1:4] = Qh[0] * u
    Qh[4] += 0.5 * Qh[0] * (u ** 2).sum(0)
    kw = dict(gamma=gamma, GM=pars["GM"], omega=omega, nu=nu, kappa=nu, T_top=pars["chi_o"])
    pf = physics(**kw)
    dtf = mf.stable_dt(pf, Qh, cfl)
    if every % 2:
        raise ValueError("the coarse run takes twice the fine step: `every` must be even")
    steps_c, dtc = every // 2, 2.0 * dtf
    Q = torch.from_numpy(Qh).cuda()
    snaps, times = resolved_snapshots(mf, pf, Q, dtf, n_spinup, n_snap, every)
    finite = bool(torch.isfinite(Q).all())
    report = {"hexes": mf.n_elems, "fine_points": mf.n_solpts, "coarse_points": mc.n_solpts, "dt_fine": dtf,
              "t_range": (times[0], times[-1]), "resolved_finite": finite}
    if not finite:
        raise RuntimeError("resolved run became non-finite")
    X, Y = samples(mf, mc, pf, snaps[:n_train], gamma)
    norm = normalisation(X, Y)
    p0 = mlp_init(seed) if params0 is None else params0
    t0 = time.perf_counter()
    P, losses = train(X, Y, norm, p0, iters, batch, seed, lr=lr)
    torch.cuda.synchronize()
    report.update(samples=int(X.shape[0]), train_seconds=time.perf_counter() - t0,
                  loss_start=float(losses[:20].mean()), loss_end=float(losses[-50:].mean()))
    model = pack_or_none(P, norm)
    report["model"], report["params"], report["norm"] = model, P, norm
    pcl = closure_physics(kw, model) if model is not None else None
    pplain = physics(**kw)
    Qb0, tau0 = filter_to_coarse(mf, mc, gamma, snaps[n_train])
    if pcl is not None:
        report["r2_heldout"], _ = apriori_r2(mc, pcl, Qb0, tau0)
    refs = [filter_to_coarse(mf, mc, gamma, s)[0] for s in snaps[n_train + 1:]]
    diag = ShellDiagnostics(mc, ri, ro, top_depth=(ro - ri) / radial_n)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    errs = judged_runs(mc, diag, pplain, pcl, Qb0, refs, dtc, steps_c, gamma)
    torch.cuda.synchronize()
    report["judge_seconds"] = time.perf_counter() - t0
    report["errors"] = errs
    report["context"] = dict(mesh=mc, diag=diag, phys_kwargs=kw, start=Qb0, refs=refs, dt=dtc, steps=steps_c)
    report["use_closure"] = choose(errs["closure"], errs["plain"], closure_finite=errs["closure"] is not None)
    return report


def cost_per_time(panel_n, radial_n, beta=0.7, order_fine=6, order_coarse=3, steps=4, cfl=0.3, seed=0,
                  kernel_times=False):
    """GPU seconds per unit simulated time of the resolved run (order_fine)
    and of the coarse run (order_coarse) without and with the fused closure
    (a seeded untrained network: the arithmetic does not depend on the
    weights), on one shell mesh; the coarse run takes
    order_fine / order_coarse times the fine step.  Timed with CUDA events
    around `steps` steps after one warm-up step."""
    from chorus_inputs import mlp_init, random_velocity, uniform_noise
    from . import chorus_mesh_create
    torch = _torch()
    ri, ro = beta / (1.0 - beta), 1.0 / (1.0 - beta)
    out = {}
    dtf = None
    for name, order in (("resolved", order_fine), ("plain", order_coarse), ("closure", order_coarse)):
        m = chorus_mesh_create(panel_n, radial_n, order, ri, ro).upload()
        Qh, pars = m.init_polytrope(beta, 1.0, noise=uniform_noise(m.n_solpts, seed), amp=1e-3)
        xyz, _ = m.solpts()
        u = random_velocity(xyz, seed + 1, amp=0.1)
        Qh[1:4] = Qh[0] * u
        Qh[4] += 0.5 * Qh[0] * (u ** 2).sum(0)
        kw = dict(GM=pars["GM"], omega=0.5, nu=1e-3, kappa=1e-3, T_top=pars["chi_o"])
        if name == "closure":
            P = torch.from_numpy(mlp_init(seed).astype(np.float32)).cuda()
            norm = torch.cat([torch.zeros(20), torch.ones(20), torch.zeros(15), torch.full((15,), 1e-3)])
            ph = closure_physics(kw, chorus_closure_pack(P, norm.float().cuda()))
        else:
            ph = physics(**kw)
        if dtf is None:
            dtf = m.stable_dt(ph, Qh, cfl)
        dt = dtf * order_fine / order
        Q = torch.from_numpy(Qh).cuda()
        ws = m.workspace(ph)
        chorus_rk_step(m, ph, Q, dt, 1, ws)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        chorus_rk_step(m, ph, Q, dt, steps, ws)
        b.record()
        torch.cuda.synchronize()
        sec = a.elapsed_time(b) * 1e-3
        out[name] = {"points": m.n_solpts, "dt": dt, "seconds_per_step": sec / steps,
                     "seconds_per_time": sec / (steps * dt), "dof_updates_per_s": m.n_solpts * steps / sec}
        if kernel_times:
            from . import chorus_kernel_timing, chorus_kernel_times
            chorus_kernel_timing(True)
            chorus_rk_step(m, ph, Q, dt, 1, ws)
            torch.cuda.synchronize()
            chorus_kernel_timing(False)
            out[name]["kernel_ms_per_launch"] = {k: v[0] / max(v[1], 1) for k, v in chorus_kernel_times().items()}
        del Q, ws
    out["ratio_resolved_over_closure"] = out["resolved"]["seconds_per_time"] / out["closure"]["seconds_per_time"]
    return out


# ---------------------------------------------------------------------------
# the configured experiment: training data from a convecting resolved run on
# the 12,288-hex shell, judged on the 98,304-hex shell
# ---------------------------------------------------------------------------
def _log(msg):
    import sys
    print("[closure] " + msg, file=sys.stderr, flush=True)


def convecting_start(mesh, beta, n_rho, luminosity, nu, omega, seed, amp, gamma=5.0 / 3.0):
    """Almost-flux-balance background (Section 4.3) at rest, Q0, and the
    same state with a seeded entropy perturbation, Q (host arrays), with the
    physics keywords (the balanced flag is added by the callers)."""
    from chorus_inputs import uniform_noise
    Q0h, pars = mesh.init_afb(beta, n_rho, luminosity, nu, gamma=gamma)
    Qh, _ = mesh.init_afb(beta, n_rho, luminosity, nu, gamma=gamma, noise=uniform_noise(mesh.n_solpts, seed),
                          amp=amp)
    kw = dict(gamma=gamma, GM=pars["GM"], omega=omega, nu=nu, kappa=nu, T_top=pars["T_top"],
              F_bottom=pars["F_bottom"])
    return Q0h, Qh, kw


def kinetic_energy(Q, wJ):
    """Volume integral of rho |u|^2 / 2 (device state, device weights)."""
    return float((0.5 * (Q[1:4] ** 2).sum(0) / Q[0] * wJ).sum())


def balanced_run(mesh, kw, Q0, Q, t_end, cfl, precision, label, chunks=12):
    """Advance Q (device) in balanced mode about Q0 to time t_end, the time
    step recomputed from the state at every chunk; logs the kinetic energy.
    Returns the time reached."""
    from . import CHORUS_BALANCED, CHORUS_FP64, chorus_set_background
    torch = _torch()
    phys = physics(precision=precision, flags=CHORUS_BALANCED, **kw)
    ws = mesh.workspace(phys)
    chorus_set_background(mesh, phys, Q0, ws)
    _, wJ = mesh.solpts()
    wJd = torch.from_numpy(wJ).to(Q.device)
    t = 0.0
    while t < t_end * (1.0 - 1e-12):
        dt = mesh.stable_dt(phys, Q.cpu().numpy(), cfl)
        n = max(1, int(math.ceil(min(t_end / chunks, t_end - t) / dt)))
        chorus_rk_step(mesh, phys, Q, dt, n, ws)
        t += n * dt
        ke = kinetic_energy(Q, wJd)
        vmax = float((((Q[1:4] / Q[0]) ** 2).sum(0)).max().sqrt())
        _log("%s: t = %.2f (dt %.2e), kinetic energy %.3e, max |u| %.3f" % (label, t, dt, ke, vmax))
        if not math.isfinite(ke):
            raise RuntimeError("%s became non-finite at t = %.2f" % (label, t))
    del ws
    return t


def configured_experiment(beta=0.73, n_rho=3.0, omega=0.5, nu=5e-5, luminosity=1e-4, amp=1e-3,
                          data_mesh=(16, 8), judge_mesh=(32, 16), order_fine=6, order_coarse=3,
                          t_spin=24.0, n_snap=13, snap_every=0.8, iters=6000, batch=4096, lr=1e-3,
                          coarse_steps=1000, n_ref=10, cfl=0.3, seed=1, gamma=5.0 / 3.0, spin_precision=None):
    """The closure experiment at the configured sizes.

    Data (12,288 hexes): a resolved order-6 run of the almost-flux-balance
    background (Section 4.3; Sun-like: beta 0.73, 3 density scale heights,
    Omega 0.5, nu = kappa = 5e-5, luminosity L) in balanced mode, from a
    seeded entropy perturbation, spun up to t_spin (convecting), then n_snap
    snapshots snap_every apart, each filtered to order 3 (331,776 samples
    per snapshot); normalisation and mini-batch Adam.
    Judged run (98,304 hexes): the same set-up at order 6 (another seed) spun
    up to t_spin and filtered to order 3 as the common start; the resolved
    run continues 2 coarse_steps steps (reference states filtered to order 3
    every 2 coarse_steps / n_ref steps), the order-3 runs without and with
    the closure take coarse_steps steps of twice the fine step; errors of
    the kinetic-energy spectrum over the outer element layer and of the
    mean radial profiles, time-averaged over the n_ref reference times;
    cost per unit simulated time of the resolved and the closure runs.
    Returns a JSON-ready report."""
    import time
    from chorus_inputs import mlp_init
    from . import CHORUS_BALANCED, CHORUS_FP64, CHORUS_MIXED, chorus_mesh_create, chorus_set_background
    torch = _torch()
    spin_precision = CHORUS_MIXED if spin_precision is None else spin_precision
    ri, ro = beta / (1.0 - beta), 1.0 / (1.0 - beta)
    report = {"config": dict(beta=beta, n_rho=n_rho, omega=omega, nu=nu, luminosity=luminosity, amp=amp,
                             data_mesh=data_mesh, judge_mesh=judge_mesh, t_spin=t_spin, n_snap=n_snap,
                             snap_every=snap_every, iters=iters, batch=batch, coarse_steps=coarse_steps,
                             n_ref=n_ref, cfl=cfl, seed=seed)}
    t_start = time.perf_counter()
    # ---- training data on the 12,288-hex shell
    mf = chorus_mesh_create(data_mesh[0], data_mesh[1], order_fine, ri, ro).upload()
    mc = chorus_mesh_create(data_mesh[0], data_mesh[1], order_coarse, ri, ro).upload()
    Q0h, Qh, kw = convecting_start(mf, beta, n_rho, luminosity, nu, omega, seed, amp, gamma)
    Q0 = torch.from_numpy(Q0h).cuda()
    Q = torch.from_numpy(Qh).cuda()
    _log("data run: %d hexes, order %d (%d points)" % (mf.n_elems, order_fine, mf.n_solpts))
    balanced_run(mf, kw, Q0, Q, t_spin, cfl, spin_precision, "data spin-up")
    p64 = physics(flags=CHORUS_BALANCED, **kw)
    ws = mf.workspace(p64)
    chorus_set_background(mf, p64, Q0, ws)
    dt = mf.stable_dt(p64, Q.cpu().numpy(), cfl)
    every = max(1, int(round(snap_every / dt)))
    snaps = [Q.clone()]
    for i in range(1, n_snap):
        chorus_rk_step(mf, p64, Q, dt, every, ws)
        snaps.append(Q.clone())
    if not bool(torch.isfinite(Q).all()):
        raise RuntimeError("data run became non-finite")
    _log("data run: %d snapshots, %d steps of %.2e apart" % (n_snap, every, dt))
    del ws
    X, Y = samples(mf, mc, physics(**kw), snaps, gamma)
    del snaps
    norm = normalisation(X, Y)
    t0 = time.perf_counter()
    P, losses = train(X, Y, norm, mlp_init(seed), iters, batch, seed, lr=lr)
    torch.cuda.synchronize()
    report["training"] = {"samples": int(X.shape[0]), "seconds": time.perf_counter() - t0,
                          "loss_start": float(losses[:20].mean()), "loss_end": float(losses[-50:].mean())}
    _log("training: %d samples, loss %.3f -> %.3f" % (X.shape[0], report["training"]["loss_start"],
                                                       report["training"]["loss_end"]))
    del X, Y, mf, mc, Q, Q0
    torch.cuda.empty_cache()
    model = pack_or_none(P, norm)
    # ---- judged runs on the 98,304-hex shell
    mf = chorus_mesh_create(judge_mesh[0], judge_mesh[1], order_fine, ri, ro).upload()
    mc = chorus_mesh_create(judge_mesh[0], judge_mesh[1], order_coarse, ri, ro).upload()
    Q0h, Qh, kw = convecting_start(mf, beta, n_rho, luminosity, nu, omega, seed + 1, amp, gamma)
    Q0 = torch.from_numpy(Q0h).cuda()
    Q = torch.from_numpy(Qh).cuda()
    del Q0h, Qh
    _log("judged run: %d hexes, resolved order %d (%d points), coarse order %d (%d points)" % (
        mf.n_elems, order_fine, mf.n_solpts, order_coarse, mc.n_solpts))
    balanced_run(mf, kw, Q0, Q, t_spin, cfl, spin_precision, "judged spin-up")
    Q0c, _ = filter_to_coarse(mf, mc, gamma, Q0)
    Qc, _ = filter_to_coarse(mf, mc, gamma, Q)
    p64 = physics(flags=CHORUS_BALANCED, **kw)
    ws = mf.workspace(p64)
    chorus_set_background(mf, p64, Q0, ws)
    dtf = mf.stable_dt(p64, Q.cpu().numpy(), cfl)
    fine_steps = 2 * coarse_steps
    per_ref = fine_steps // n_ref
    refs = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(n_ref):
        chorus_rk_step(mf, p64, Q, dtf, per_ref, ws)
        refs.append(filter_to_coarse(mf, mc, gamma, Q)[0])
    torch.cuda.synchronize()
    wall_fine = time.perf_counter() - t0
    if not bool(torch.isfinite(Q).all()):
        raise RuntimeError("resolved judged run became non-finite")
    _log("resolved reference: %d steps of %.2e in %.1f s" % (fine_steps, dtf, wall_fine))
    del ws, Q, Q0
    torch.cuda.empty_cache()
    diag = ShellDiagnostics(mc, ri, ro, top_depth=(ro - ri) / judge_mesh[1])
    refs_h = [r.cpu().numpy() for r in refs]
    del refs
    errors, walls = {}, {}
    for name, mdl in (("plain", None), ("closure", model)):
        if name == "closure" and mdl is None:
            errors[name] = None
            continue
        ph = closure_physics(dict(kw, flags=CHORUS_BALANCED), mdl)
        wsc = mc.workspace(ph)
        chorus_set_background(mc, ph, Q0c, wsc)
        q = Qc.clone()
        errs, wall = [], 0.0
        for i in range(n_ref):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            chorus_rk_step(mc, ph, q, 2.0 * dtf, per_ref // 2, wsc)
            torch.cuda.synchronize()
            wall += time.perf_counter() - t0
            if not bool(torch.isfinite(q).all()):
                errs = None
                break
            errs.append(judge_errors(diag, q.cpu().numpy(), refs_h[i], gamma))
        errors[name] = mean_errors(errs) if errs else None
        walls[name] = wall
        _log("%s run: %s" % (name, errors[name]))
        del wsc, q
    sim_time = fine_steps * dtf
    report["judged"] = {"resolved_points": mf.n_solpts, "coarse_points": mc.n_solpts, "dt_fine": dtf,
                        "fine_steps": fine_steps, "coarse_steps": coarse_steps, "simulated_time": sim_time,
                        "errors": errors,
                        "worst": {k: (score(v) if v else None) for k, v in errors.items()},
                        "seconds_per_unit_time": {"resolved": wall_fine / sim_time,
                                                  **{k: v / sim_time for k, v in walls.items()}}}
    if "closure" in walls:
        report["judged"]["cost_ratio_resolved_over_closure"] = wall_fine / walls["closure"]
    use = choose(errors.get("closure"), errors["plain"], closure_finite=errors.get("closure") is not None)
    report["use_closure"] = bool(use)
    report["within_5_percent"] = bool(errors.get("closure") is not None and score(errors["closure"]) <= 0.05)
    report["seconds"] = time.perf_counter() - t_start
    return report


if __name__ == "__main__":
    import argparse
    import json
    ap = argparse.ArgumentParser(description="the closure experiment at the configured sizes (one JSON line)")
    ap.add_argument("--t-spin", type=float, default=24.0)
    ap.add_argument("--iters", type=int, default=6000)
    ap.add_argument("--coarse-steps", type=int, default=1000)
    ap.add_argument("--data-mesh", default="16,8")
    ap.add_argument("--judge-mesh", default="32,16")
    ap.add_argument("--luminosity", type=float, default=1e-4)
    ap.add_argument("--amp", type=float, default=1e-3)
    a = ap.parse_args()
    rep = configured_experiment(t_spin=a.t_spin, iters=a.iters, coarse_steps=a.coarse_steps,
                                data_mesh=tuple(int(v) for v in a.data_mesh.split(",")),
                                judge_mesh=tuple(int(v) for v in a.judge_mesh.split(",")),
                                luminosity=a.luminosity, amp=a.amp)
    print(json.dumps(rep), flush=True)
