"""Halo depth of one residual evaluation (the basis of how the path would
shard by element partition, Section 3's compact stencil).

The SD residual of an element set A depends on the state of A, of its face
neighbours N1(A) and, through the neighbours' BR1 gradients (viscous terms),
of their neighbours N2(A): two exchanges per stage.  With the state set to
NaN outside N2(A), the residual on A is bitwise unchanged, and with NaN
outside N1(A) it is NaN.  Without viscosity and diffusion one exchange
suffices: a different (valid) state outside N1(A) leaves the residual on A
bitwise unchanged (the diffusive terms still multiply the gradients by zero
coefficients, so NaN there would show through), while a different state
outside A changes it.  Checked on the oracle (CPU) and on both GPU paths.
"""
import numpy as np
import pytest

from chorus_inputs import cubed_sphere_shell, uniform_noise


def _case(oracle_mod):
    beta = 0.7
    ri, ro = beta / (1 - beta), 1 / (1 - beta)
    m = cubed_sphere_shell(5, 2, ri, ro)
    om = oracle_mod.OracleMesh(m, 3)
    Q0, pars = om.polytrope(beta, 1.0)
    Q, _ = om.polytrope(beta, 1.0, noise=uniform_noise(om.n_solpts, 21), amp=1e-3)
    rng = np.random.default_rng(22)
    Q[1:4] = 1e-2 * Q[0] * rng.uniform(-1, 1, size=Q[1:4].shape)
    Q[4] += 0.5 * (Q[1:4] ** 2).sum(0) / Q[0]
    ne, _, _ = om.faces()
    A = np.arange(om.E) < 15                   # a patch of 15 elements

    def grow(S):
        T = S.copy()
        for e in np.nonzero(S)[0]:
            for nb in ne[e]:
                if nb >= 0:
                    T[nb] = True
        return T
    N1 = grow(A)
    N2 = grow(N1)
    assert N1.sum() > A.sum() and N2.sum() > N1.sum() and N2.sum() < om.E
    return m, om, pars, Q0, Q, A, N1, N2


def _blank(Q, keep):
    Qb = Q.copy()
    Qb[:, ~keep, :] = np.nan
    return Qb


def _other(Q, keep):
    """A different valid state outside `keep` (density and energy +5 %)."""
    Qo = Q.copy()
    Qo[:, ~keep, :] *= 1.05
    return Qo


def test_oracle_halo_depth(oracle_mod):
    m, om, pars, Q0, Q, A, N1, N2 = _case(oracle_mod)
    visc = oracle_mod.phys(GM=pars["GM"], omega=1.0, nu=1e-3, kappa=1e-3, T_top=pars["chi_o"])
    invisc = oracle_mod.phys(GM=pars["GM"], omega=1.0)
    R = om.residual(visc, Q)
    assert np.array_equal(om.residual(visc, _blank(Q, N2))[:, A], R[:, A])
    assert np.isnan(om.residual(visc, _blank(Q, N1))[:, A]).any()
    Ri = om.residual(invisc, Q)
    assert np.array_equal(om.residual(invisc, _other(Q, N1))[:, A], Ri[:, A])
    assert not np.array_equal(om.residual(invisc, _other(Q, A))[:, A], Ri[:, A])


@pytest.mark.gpu
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_gpu_halo_depth(oracle_mod, precision):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1503_00834_amd as ch
    m, om, pars, Q0, Q, A, N1, N2 = _case(oracle_mod)
    prec = ch.CHORUS_MIXED if precision == "mixed" else ch.CHORUS_FP64
    cm = ch.mesh_from_arrays(m, 3).upload()

    def residual(phys, Qh):
        ws = cm.workspace(phys)
        if prec == ch.CHORUS_MIXED:
            ch.chorus_set_background(cm, phys, torch.from_numpy(np.ascontiguousarray(Q0.reshape(5, -1))).cuda(), ws)
        Qd = torch.from_numpy(np.ascontiguousarray(Qh.reshape(5, -1))).cuda()
        R = torch.empty_like(Qd)
        ch.chorus_sd_residual(cm, phys, Qd, R, ws)
        torch.cuda.synchronize()
        return R.cpu().numpy().reshape(5, om.E, om.np)

    visc = ch.physics(GM=pars["GM"], omega=1.0, nu=1e-3, kappa=1e-3, T_top=pars["chi_o"], precision=prec)
    invisc = ch.physics(GM=pars["GM"], omega=1.0, precision=prec)
    R = residual(visc, Q)
    assert np.isfinite(R).all()
    assert np.array_equal(residual(visc, _blank(Q, N2))[:, A], R[:, A])
    assert np.isnan(residual(visc, _blank(Q, N1))[:, A]).any()
    Ri = residual(invisc, Q)
    assert np.array_equal(residual(invisc, _other(Q, N1))[:, A], Ri[:, A])
    assert not np.array_equal(residual(invisc, _other(Q, A))[:, A], Ri[:, A])
