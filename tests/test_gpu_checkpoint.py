"""Checkpoint and resume.

Between calls of `chorus_rk_step` the solver state is the FP64 state Q
([5][E][N^3], caller-owned) together with dt and the step count, which are
call arguments; on the mixed path the background Q0 that
`chorus_set_background` stored in the workspace is state too.  A run that
is stopped, written to disk, read back into fresh device buffers, a fresh
mesh handle and a fresh workspace therefore continues exactly:

* FP64 path: bit-identical to the uninterrupted run (both integrators);
* mixed path: the perturbation P = Q - Q0 is carried in FP64 across the
  steps of one call and re-formed from Q at the start of the next, so a
  restart rounds P once through Q = Q0 + P (half an ulp of Q).  The resumed
  run agrees with the uninterrupted one to that rounding, carried through
  the FP32 residual.

The oracle is checked the same way on the CPU (stop, save, load, continue).
"""
import os

import numpy as np
import pytest

from chorus_inputs import cubed_sphere_shell, uniform_noise
from test_gpu_parity import shell_case


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def ch(torch_dev):
    import paper_1503_00834_amd as ch
    return ch


def _save_load(tmp_path, name, arrays):
    """Round trip through .npy files (what a checkpoint writes and reads)."""
    out = []
    for i, a in enumerate(arrays):
        f = os.path.join(str(tmp_path), "%s_%d.npy" % (name, i))
        np.save(f, a)
        out.append(np.load(f))
    return out


def test_oracle_resume_is_exact(oracle_mod, tmp_path):
    m = cubed_sphere_shell(2, 1, 7.0 / 3.0, 10.0 / 3.0)
    om = oracle_mod.OracleMesh(m, 3)
    Q, pars = om.polytrope(0.7, 1.0, noise=uniform_noise(om.n_solpts, 4), amp=1e-3)
    op = oracle_mod.phys(GM=pars["GM"], omega=1.0, nu=1e-3, kappa=1e-3)
    dt = 0.02
    for step in (om.rk3, om.ssp54):
        whole = step(op, Q, dt, 3)
        (half,) = _save_load(tmp_path, step.__name__, [step(op, Q, dt, 1)])
        assert np.array_equal(step(op, half, dt, 2), whole), step.__name__


@pytest.mark.gpu
@pytest.mark.parametrize("integrator", ["rk3", "ssp54"])
def test_fp64_resume_is_bit_identical(ch, oracle_mod, torch_dev, tmp_path, integrator):
    torch = torch_dev
    m, om, Q, phys = shell_case(oracle_mod, ch, 4, 3, 3, amp=1e-3)
    phys.integrator = ch.CHORUS_SSPRK3 if integrator == "rk3" else ch.CHORUS_SSPRK54
    dt, n1, n2 = 0.02, 4, 3

    def dev(a):
        return torch.from_numpy(np.ascontiguousarray(a.reshape(5, -1))).cuda()

    cm = ch.mesh_from_arrays(m, 3).upload()
    Qd = dev(Q)
    ch.chorus_rk_step(cm, phys, Qd, dt, n1 + n2, cm.workspace(phys))
    torch.cuda.synchronize()
    whole = Qd.cpu().numpy()
    # stop after n1 steps and write the state out
    Qd = dev(Q)
    ch.chorus_rk_step(cm, phys, Qd, dt, n1, cm.workspace(phys).fill_(255))
    torch.cuda.synchronize()
    (saved,) = _save_load(tmp_path, "fp64_" + integrator, [Qd.cpu().numpy()])
    del cm, Qd
    # a fresh mesh handle, device buffers and NaN-filled workspace
    cm2 = ch.mesh_from_arrays(m, 3).upload()
    Qd = dev(saved)
    ch.chorus_rk_step(cm2, phys, Qd, dt, n2, cm2.workspace(phys).fill_(255))
    torch.cuda.synchronize()
    resumed = Qd.cpu().numpy()
    assert np.isfinite(resumed).all()
    assert np.array_equal(resumed, whole)


@pytest.mark.gpu
def test_mixed_resume_matches_to_rounding(ch, oracle_mod, torch_dev, tmp_path):
    torch = torch_dev
    beta, n_rho = 0.7, 1.0
    ri, ro = beta / (1 - beta), 1 / (1 - beta)
    m = cubed_sphere_shell(4, 3, ri, ro)
    om = oracle_mod.OracleMesh(m, 4)
    Q0, pars = om.polytrope(beta, n_rho)
    Q, _ = om.polytrope(beta, n_rho, noise=uniform_noise(om.n_solpts, 6), amp=1e-3)
    rng = np.random.default_rng(7)
    Q[1:4] = 1e-3 * Q[0] * rng.uniform(-1, 1, size=Q[1:4].shape)
    Q[4] += 0.5 * (Q[1:4] ** 2).sum(0) / Q[0]
    phys = ch.physics(GM=pars["GM"], omega=1.0, nu=1e-3, kappa=1e-3, T_top=pars["chi_o"], F_bottom=0.01,
                      precision=ch.CHORUS_MIXED)
    dt, n1, n2 = 0.01, 4, 3

    def dev(a):
        return torch.from_numpy(np.ascontiguousarray(a.reshape(5, -1))).cuda()

    cm = ch.mesh_from_arrays(m, 4).upload()
    ws = cm.workspace(phys)
    ch.chorus_set_background(cm, phys, dev(Q0), ws)
    Qd = dev(Q)
    ch.chorus_rk_step(cm, phys, Qd, dt, n1 + n2, ws)
    torch.cuda.synchronize()
    whole = Qd.cpu().numpy()
    Qd = dev(Q)
    ch.chorus_rk_step(cm, phys, Qd, dt, n1, ws)
    torch.cuda.synchronize()
    saved, bg = _save_load(tmp_path, "mixed", [Qd.cpu().numpy(), Q0.reshape(5, -1)])
    del cm, ws, Qd
    cm2 = ch.mesh_from_arrays(m, 4).upload()
    ws2 = cm2.workspace(phys).fill_(255)
    ch.chorus_set_background(cm2, phys, dev(bg), ws2)
    Qd = dev(saved)
    ch.chorus_rk_step(cm2, phys, Qd, dt, n2, ws2)
    torch.cuda.synchronize()
    resumed = Qd.cpu().numpy()
    assert np.isfinite(resumed).all()
    start = Q.reshape(5, -1)
    for v in range(5):
        change = np.linalg.norm(whole[v] - start[v])
        diff = np.linalg.norm(resumed[v] - whole[v])
        # the restart moves P by at most half an ulp of Q
        assert np.abs(resumed[v] - whole[v]).max() <= 1e-6 * np.abs(whole[v] - start[v]).max() + \
            8 * np.spacing(np.abs(whole[v]).max()), v
        assert diff <= 1e-7 * change + 1e-15 * np.linalg.norm(whole[v]), (v, diff, change)
        print("mixed resume: variable %d, |resumed - whole| / |change| = %.2e" % (v, diff / change))
