"""The 331,776-hex N = 4 benchmark workload at full size against the oracle
on sampled elements.

The residual of an element depends on the state of its face neighbours and
of their neighbours only (two BR1 exchanges, `test_halo_depth.py`), one
SSP-RK3 step on six such rings.  So the oracle runs on a sub-mesh made of the
sampled elements and their rings: the faces cut at the sub-mesh's edge
become far-field boundaries, which change only the outer rings.  The GPU's
full-size results at the sampled elements are then compared with the
oracle's there, element by element, to the bounds of the smaller cases
(FP64: 1e-12 relative or twice the one-ulp sensitivity floor; mixed: the
perturbation-relative bound of `test_gpu_mixed.py`).

The state is generated here from the solution-point coordinates, the 20-node
map evaluated at the tensor Chebyshev-Gauss points; that helper and the face
matching used to grow the rings are pinned against the oracle's own
coordinates and face table on a small shell (CPU tests below).
"""
import math

import numpy as np
import pytest

from chorus_inputs import (CONFIGS, HEX20_LOCAL, Hex20Mesh, cubed_sphere_shell, shell_params_from_config,
                           uniform_noise)

GAMMA = 5.0 / 3.0
# corner nodes (i + 2j + 4k) of faces xi=0, xi=1, eta=0, eta=1, zeta=0, zeta=1
FACE_CORNERS = [[0, 2, 4, 6], [1, 3, 5, 7], [0, 1, 4, 5], [2, 3, 6, 7], [0, 1, 2, 3], [4, 5, 6, 7]]


def hex20_shape(x):
    """Serendipity shape functions of the 20 nodes (HEX20_LOCAL: positions
    on the doubled lattice 0, 1, 2 of the reference cube) at local points x
    in [0, 1]^3, [n][3] -> [n][20]."""
    a = 2.0 * np.asarray(x, dtype=np.float64) - 1.0
    nodes = np.asarray(HEX20_LOCAL, dtype=np.float64) - 1.0
    out = np.empty((a.shape[0], 20))
    for n, c in enumerate(nodes):
        f = [(1.0 + a[:, d] * c[d]) if c[d] != 0.0 else (1.0 - a[:, d] ** 2) for d in range(3)]
        if np.all(c != 0.0):
            out[:, n] = f[0] * f[1] * f[2] * ((a * c).sum(1) - 2.0) / 8.0
        else:
            out[:, n] = f[0] * f[1] * f[2] / 4.0
    return out


def hex20_solpts(m, N):
    """Solution-point coordinates [3][E N^3] (point i + N (j + N k), the
    Chebyshev-Gauss points (1 - cos((2s+1) pi / 2N)) / 2 along each axis)."""
    xs = 0.5 * (1.0 - np.cos((2.0 * np.arange(N) + 1.0) * math.pi / (2.0 * N)))
    k, j, i = np.meshgrid(xs, xs, xs, indexing="ij")
    loc = np.stack([i.ravel(), j.ravel(), k.ravel()], axis=1)
    H = hex20_shape(loc)                                   # [N^3][20]
    X = m.xyz[m.elem20]                                     # [E][20][3]
    return np.einsum("pn,enc->cep", H, X).reshape(3, -1)


def face_neighbours(m):
    """Neighbour element across each face [E][6] (-1 on boundaries), by the
    match ids of the faces' four corners."""
    E = m.n_elems
    c = m.match_id[m.elem20[:, :8]]
    keys = np.sort(np.stack([c[:, fc] for fc in FACE_CORNERS], axis=1), axis=2).reshape(-1, 4)
    order = np.lexsort(keys.T[::-1])
    s = keys[order]
    same = np.nonzero(np.all(s[1:] == s[:-1], axis=1))[0]
    nb = np.full(E * 6, -1, dtype=np.int64)
    nb[order[same]] = order[same + 1] // 6
    nb[order[same + 1]] = order[same] // 6
    return nb.reshape(E, 6)


def rings(nb, seeds, depth):
    S = np.zeros(nb.shape[0], dtype=bool)
    S[seeds] = True
    for _ in range(depth):
        n = nb[S]
        S[n[n >= 0]] = True
    return S


def sub_mesh(m, nb, S):
    """The elements S as a mesh of their own; faces to elements outside S
    become far-field boundaries (tag 3)."""
    idx = np.nonzero(S)[0]
    e20 = m.elem20[idx]
    nodes, inv = np.unique(e20, return_inverse=True)
    fbc = m.face_bc[idx].copy()
    n = nb[idx]
    fbc[(n >= 0) & ~S[np.maximum(n, 0)]] = 3
    sub = Hex20Mesh(xyz=m.xyz[nodes], elem20=inv.reshape(e20.shape).astype(np.int64),
                    face_bc=fbc.astype(np.int32), match_id=np.arange(nodes.size, dtype=np.int64))
    return sub, idx


def stratified_state(xyz, ri, ro, seed, moving=True):
    """Hotter and denser inward, a seeded density perturbation of 1e-3 and
    (when moving) a smooth velocity of amplitude 0.02."""
    r = np.sqrt((xyz ** 2).sum(0))
    T = 1.0 + 2.0 * (ro - r) / (ro - ri)
    rho = T ** 1.5 * (1.0 + 1e-3 * uniform_noise(r.size, seed))
    u = 0.02 * np.stack([np.sin(xyz[1]), np.sin(xyz[2]), np.sin(xyz[0])]) if moving else np.zeros_like(xyz)
    E = rho * T / (GAMMA - 1.0) + 0.5 * rho * (u ** 2).sum(0)
    return np.concatenate([rho[None], rho * u, E[None]])


def _small_shell():
    beta = 0.7
    return cubed_sphere_shell(3, 2, beta / (1 - beta), 1 / (1 - beta))


def test_solpts_helper_matches_oracle(oracle_mod):
    m = _small_shell()
    for N in (3, 4):
        xyz, _ = oracle_mod.OracleMesh(m, N).solpts()
        assert np.allclose(hex20_solpts(m, N), xyz, rtol=0, atol=1e-13 * np.abs(xyz).max())


def test_face_neighbours_match_oracle(oracle_mod):
    m = _small_shell()
    ne, _, _ = oracle_mod.OracleMesh(m, 3).faces()
    assert np.array_equal(face_neighbours(m), ne)


def test_sub_mesh_residual_exact_two_rings_in(oracle_mod):
    """The construction itself: on a small shell the sub-mesh residual at
    the seed elements equals the full mesh's bitwise (viscous, walls)."""
    m = _small_shell()
    ri, ro = 0.7 / 0.3, 1 / 0.3
    om = oracle_mod.OracleMesh(m, 3)
    xyz, _ = om.solpts()
    Q = stratified_state(xyz, ri, ro, 5).reshape(5, m.n_elems, -1)
    ph = oracle_mod.phys(gamma=GAMMA, GM=5.0, omega=0.5, nu=1e-3, kappa=1e-3, T_top=1.0)
    nb = face_neighbours(m)
    seeds = np.array([0, m.n_elems // 2, m.n_elems - 1])
    sub, idx = sub_mesh(m, nb, rings(nb, seeds, 2))
    assert idx.size < m.n_elems
    pos = np.searchsorted(idx, seeds)
    Rs = oracle_mod.OracleMesh(sub, 3).residual(ph, Q[:, idx])[:, pos]
    assert np.array_equal(Rs, om.residual(ph, Q)[:, seeds])
    # one ring is not enough (the neighbours' gradients see the cut faces)
    sub1, idx1 = sub_mesh(m, nb, rings(nb, seeds, 1))
    R1 = oracle_mod.OracleMesh(sub1, 3).residual(ph, Q[:, idx1])[:, np.searchsorted(idx1, seeds)]
    assert not np.array_equal(R1, Rs)


@pytest.mark.gpu
def test_full_size_sun_workload_sampled(oracle_mod):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1503_00834_amd as ch
    from test_gpu_mixed import assert_mixed
    from test_gpu_parity import assert_parity, ora_phys, perturbed_oracle, ulp_perturb
    cfg = CONFIGS["sun_332k_N4"]
    ri, ro = shell_params_from_config(cfg)
    N = cfg["order"]
    m = cubed_sphere_shell(cfg["panel_n"], cfg["radial_n"], ri, ro)
    E, NP = m.n_elems, N ** 3
    print("sun_332k_N4 sampled: %d hexes generated" % E, flush=True)
    xyz = hex20_solpts(m, N)
    Q = stratified_state(xyz, ri, ro, cfg["seed"])
    Q0 = stratified_state(xyz, ri, ro, cfg["seed"], moving=False)
    cm = ch.chorus_mesh_create(cfg["panel_n"], cfg["radial_n"], N, ri, ro).upload()
    # the library's shell is the input generator's element for element
    xl, _ = cm.solpts()
    assert np.abs(xl - xyz).max() <= 1e-12 * np.abs(xyz).max()
    nb = face_neighbours(m)
    rng = np.random.default_rng(cfg["seed"] + 17)
    inner = np.nonzero((m.face_bc == 1).any(1))[0]
    outer = np.nonzero((m.face_bc == 2).any(1))[0]
    seeds = np.unique(np.concatenate([rng.choice(inner, 3, replace=False), rng.choice(outer, 3, replace=False),
                                      rng.choice(E, 6, replace=False)]))
    Qe, Q0e = Q.reshape(5, E, NP), Q0.reshape(5, E, NP)
    kw = dict(GM=25.0, omega=cfg["omega"], nu=cfg["nu"], kappa=cfg["kappa"], kappa_r=2e-5, T_top=1.0,
              F_bottom=1e-3)
    phys = ch.physics(**kw)
    op = ora_phys(oracle_mod, phys)

    # residual (FP64): two rings
    Qd = torch.from_numpy(np.ascontiguousarray(Q)).cuda()
    R = torch.empty_like(Qd)
    ws = cm.workspace(phys)
    ch.chorus_sd_residual(cm, phys, Qd, R, ws)
    torch.cuda.synchronize()
    Rg = R.cpu().numpy().reshape(5, E, NP)[:, seeds]
    sub, idx = sub_mesh(m, nb, rings(nb, seeds, 2))
    pos = np.searchsorted(idx, seeds)
    print("residual sub-mesh: %d of %d elements" % (idx.size, E), flush=True)
    Ro = oracle_mod.OracleMesh(sub, N).residual(op, Qe[:, idx])[:, pos]
    Rp = perturbed_oracle(oracle_mod, sub, N).residual(op, ulp_perturb(Qe[:, idx]))[:, pos]
    assert_parity(Rg, Ro, Rp, "sun_332k_N4 residual (sampled)")

    # one SSP-RK3 step (FP64): six rings
    dt = 1e-3
    ch.chorus_rk_step(cm, phys, Qd, dt, 1, ws)
    torch.cuda.synchronize()
    Q1 = Qd.cpu().numpy().reshape(5, E, NP)[:, seeds]
    sub6, idx6 = sub_mesh(m, nb, rings(nb, seeds, 6))
    pos6 = np.searchsorted(idx6, seeds)
    print("RK3 sub-mesh: %d of %d elements" % (idx6.size, E), flush=True)
    Qs = Qe[:, idx6]
    Q1o = oracle_mod.OracleMesh(sub6, N).rk3(op, Qs, dt, 1)[:, pos6]
    Q1p = perturbed_oracle(oracle_mod, sub6, N).rk3(op, ulp_perturb(Qs), dt, 1)[:, pos6]
    q0 = Qe[:, seeds]
    assert_parity(Q1 - q0, Q1o - q0, Q1p - q0, "sun_332k_N4 rk3 (sampled)")

    # mixed residual against R(Q) - R(Q0): two rings
    mphys = ch.physics(precision=ch.CHORUS_MIXED, **kw)
    mws = cm.workspace(mphys)
    ch.chorus_set_background(cm, mphys, torch.from_numpy(np.ascontiguousarray(Q0)).cuda(), mws)
    Qd = torch.from_numpy(np.ascontiguousarray(Q)).cuda()
    ch.chorus_sd_residual(cm, mphys, Qd, R, mws)
    torch.cuda.synchronize()
    Rm = R.cpu().numpy().reshape(5, E, NP)[:, seeds]
    Rb = oracle_mod.OracleMesh(sub, N).residual(op, Q0e[:, idx])[:, pos]
    assert_mixed(Rm.reshape(5, -1), Ro.reshape(5, -1), Rb.reshape(5, -1), "sun_332k_N4 mixed residual (sampled)")
