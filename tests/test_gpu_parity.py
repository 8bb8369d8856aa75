"""GPU parity of the FP64 SD residual and SSP-RK3 update against the CPU
oracle, through the C-ABI, element by element.

Tolerance (FP64 mode): per conserved variable v, in the L2 norm over all
points and in the max norm,
    ||R_gpu,v - R_oracle,v|| <= max(1e-12 ||R_oracle,v||, K * floor_v)
where floor_v is the oracle's own rounding sensitivity in the same norm:
the change of its output when every state value and every node coordinate
is perturbed by one unit in the last place (random signs).  The GPU library
computes the same geometry, 1D operators and fluxes with its own code, a
different summation order and fused multiply-adds: rounding-level
perturbations of that size.  K = 2 unless a case lists its measured factor
(FLOOR_FACTOR below).  Every case prints its achieved error relative to the
reference norm and to the floor, and which bound applied.
"""
import numpy as np
import pytest

from chorus_inputs import box_mesh, cubed_sphere_shell, two_element_mesh, uniform_noise

pytestmark = pytest.mark.gpu


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


def ulp_perturb(Q, seed=7):
    rng = np.random.default_rng(seed)
    return Q * (1.0 + np.finfo(np.float64).eps * rng.choice([-1.0, 1.0], size=Q.shape))


def perturbed_oracle(oracle_mod, mesh, N, seed=11):
    """Oracle on the same mesh with every node coordinate moved by one ulp."""
    import copy
    m2 = copy.deepcopy(mesh)
    m2.xyz = ulp_perturb(m2.xyz, seed)
    return oracle_mod.OracleMesh(m2, N)


FLOOR_FACTOR = 2.0


def assert_parity(R_gpu, R_ref, R_pert, what, rel=1e-12, factor=None):
    """Per variable: L2 and max-norm error within max(rel * |R_ref|,
    factor * floor) of the same norm; prints the achieved errors."""
    factor = FLOOR_FACTOR if factor is None else factor
    R_gpu = R_gpu.reshape(5, -1)
    R_ref = R_ref.reshape(5, -1)
    dp = R_pert.reshape(5, -1) - R_ref
    d = R_gpu - R_ref
    fails = []
    for v in range(5):
        for norm, f in (("L2", lambda a: float(np.linalg.norm(a))), ("max", lambda a: float(np.abs(a).max()))):
            err, ref, floor = f(d[v]), f(R_ref[v]), f(dp[v])
            tol = max(rel * ref, factor * floor, 1e-300)
            bound = "1e-12 rel" if rel * ref >= factor * floor else "%g x floor" % factor
            print("%s var %d %s: err/ref %.2e err/floor %.2f (bound %s)" % (
                what, v, norm, err / max(ref, 1e-300), err / max(floor, 1e-300), bound))
            if not err <= tol:
                fails.append("%s var %d %s: err %.3e tol %.3e (ref %.3e floor %.3e)" % (
                    what, v, norm, err, tol, ref, floor))
    assert not fails, "; ".join(fails)


def ora_phys(oracle_mod, p):
    return oracle_mod.phys(gamma=p.gamma, R_gas=p.R_gas, GM=p.GM, omega=p.omega, nu=p.nu, kappa=p.kappa,
                           kappa_r=p.kappa_r, T_top=p.T_top, F_bottom=p.F_bottom,
                           bc_state=tuple(p.bc_state), kappa_r1=p.kappa_r1, kappa_r2=p.kappa_r2)


def gpu_residual(ch, torch, cm, phys, Q):
    Qd = torch.from_numpy(np.ascontiguousarray(Q.reshape(5, -1))).cuda()
    R = torch.empty_like(Qd)
    ws = cm.workspace(phys)
    ch.chorus_sd_residual(cm, phys, Qd, R, ws)
    torch.cuda.synchronize()
    return R.cpu().numpy()


def shell_case(oracle_mod, ch, panel_n, radial_n, N, beta=0.7, n_rho=1.0, amp=1e-2, seed=0):
    ri, ro = beta / (1 - beta), 1 / (1 - beta)
    m = cubed_sphere_shell(panel_n, radial_n, ri, ro)
    om = oracle_mod.OracleMesh(m, N)
    Q, pars = om.polytrope(beta, n_rho, noise=uniform_noise(om.n_solpts, seed), amp=amp)
    # add a seeded velocity field so that every flux term is exercised
    rng = np.random.default_rng(seed + 1)
    Q[1:4] = 0.05 * Q[0] * rng.uniform(-1, 1, size=Q[1:4].shape)
    Q[4] += 0.5 * (Q[1:4] ** 2).sum(0) / Q[0]
    phys = ch.physics(GM=pars["GM"], omega=1.0, nu=1e-3, kappa=1e-3, kappa_r=2e-4, T_top=pars["chi_o"],
                      F_bottom=0.01)
    return m, om, Q, phys


@pytest.mark.parametrize("N", [3, 4])
def test_residual_parity_shell(ch, oracle_mod, torch_dev, N):
    m, om, Q, phys = shell_case(oracle_mod, ch, 3, 2, N)
    cm = ch.mesh_from_arrays(m, N).upload()
    R = gpu_residual(ch, torch_dev, cm, phys, Q)
    op = ora_phys(oracle_mod, phys)
    Rp = perturbed_oracle(oracle_mod, m, N).residual(op, ulp_perturb(Q))
    assert_parity(R, om.residual(op, Q), Rp, "shell N=%d" % N)


@pytest.mark.parametrize("N", [3, 4])
def test_residual_parity_radial_kappa_r(ch, oracle_mod, torch_dev, N):
    """Radiative diffusivity varying with radius (solar case, Section 7.4):
    kappa_r(r) = kappa_r + kappa_r1 r + kappa_r2 r^2 at each flux point's
    radius; the radial terms change the residual by far more than the
    tolerance."""
    m, om, Q, phys = shell_case(oracle_mod, ch, 3, 2, N)
    phys.kappa_r1, phys.kappa_r2 = 3e-4, 1e-4
    cm = ch.mesh_from_arrays(m, N).upload()
    R = gpu_residual(ch, torch_dev, cm, phys, Q)
    op = ora_phys(oracle_mod, phys)
    Rr = om.residual(op, Q)
    Rp = perturbed_oracle(oracle_mod, m, N).residual(op, ulp_perturb(Q))
    assert_parity(R, Rr, Rp, "radial kappa_r N=%d" % N)
    phys.kappa_r1, phys.kappa_r2 = 0.0, 0.0
    R0 = om.residual(ora_phys(oracle_mod, phys), Q).reshape(5, -1)
    assert np.linalg.norm(Rr.reshape(5, -1)[4] - R0[4]) > 1e-6 * np.linalg.norm(R0[4])


def test_negative_radial_kappa_r_rejected(ch, oracle_mod, torch_dev):
    """kappa_r(r) negative somewhere on the mesh: CHORUS_EINVAL, nothing run."""
    m, om, Q, phys = shell_case(oracle_mod, ch, 2, 1, 3)
    cm = ch.mesh_from_arrays(m, 3).upload()
    phys.kappa_r, phys.kappa_r1 = 1e-4, -1e-3  # negative near the outer wall
    with pytest.raises(ch.ChorusError) as ei:
        gpu_residual(ch, torch_dev, cm, phys, Q)
    assert ei.value.status == -1


def test_residual_parity_c1_config(ch, oracle_mod, torch_dev):
    """The 288-hex, N=3 shell of the plain FP64 configuration."""
    m, om, Q, phys = shell_case(oracle_mod, ch, 4, 3, 3, amp=1e-4)
    cm = ch.mesh_from_arrays(m, 3).upload()
    R = gpu_residual(ch, torch_dev, cm, phys, Q)
    op = ora_phys(oracle_mod, phys)
    Rp = perturbed_oracle(oracle_mod, m, 3).residual(op, ulp_perturb(Q))
    assert_parity(R, om.residual(op, Q), Rp, "C1")


@pytest.mark.parametrize("N", [2, 3, 4, 5, 6])
def test_residual_parity_periodic_box_all_orders(ch, oracle_mod, torch_dev, N):
    m = box_mesh(3, 3, 3, periodic=(True,) * 3, curve=0.03)
    om = oracle_mod.OracleMesh(m, N)
    xyz, _ = om.solpts()
    x, y, z = xyz
    Q = np.stack([1 + 0.2 * np.sin(2 * np.pi * (x + y)), 0.3 + 0.1 * np.cos(2 * np.pi * z),
                  -0.2 + 0.05 * np.sin(2 * np.pi * x), 0.1 * np.cos(2 * np.pi * y), 2.5 + 0.1 * np.sin(2 * np.pi * z)])
    phys = ch.physics(GM=1.0, omega=0.5, nu=1e-2, kappa=1e-2, kappa_r=1e-3)
    cm = ch.mesh_from_arrays(m, N).upload()
    R = gpu_residual(ch, torch_dev, cm, phys, Q)
    op = ora_phys(oracle_mod, phys)
    Qo = Q.reshape(5, om.E, om.np)
    Rp = perturbed_oracle(oracle_mod, m, N).residual(op, ulp_perturb(Qo))
    assert_parity(R, om.residual(op, Qo), Rp, "box N=%d" % N)



@pytest.mark.parametrize("N", [3, 4])
def test_linear_velocity_and_pressure_euler_exact_gpu(ch, oracle_mod, torch_dev, N):
    """Closed-form pin of the FP64 kernels, no oracle values: u = U + A x,
    p = p0 + b.x, uniform rho on an affine box (every flux at most cubic,
    exact at N >= 3), so the residual of the interior element is the exact
    Euler dQ/dt of Section 2 (the same state as the oracle's pin)."""
    m = box_mesh(3, 3, 3, lengths=(1.0, 1.2, 0.9), origin=(-0.5, -0.6, -0.45))
    cm = ch.mesh_from_arrays(m, N).upload()
    xyz, _ = cm.solpts()
    A = np.array([[0.3, -0.2, 0.5], [0.1, -0.4, 0.25], [-0.3, 0.2, 0.15]])
    U = np.array([0.2, -0.1, 0.05])
    b = np.array([0.3, -0.5, 0.2])
    rho, p0, gam = 1.3, 2.0, 5.0 / 3.0
    u = U[:, None] + A @ xyz
    p = p0 + b @ xyz
    E = p / (gam - 1) + 0.5 * rho * (u ** 2).sum(0)
    Q = np.concatenate([np.full((1, xyz.shape[1]), rho), rho * u, E[None]])
    R = gpu_residual(ch, torch_dev, cm, ch.physics(gamma=gam), Q)
    trA = np.trace(A)
    gradE = b[:, None] / (gam - 1) + rho * (A.T @ u)
    exact = np.concatenate([np.full((1, xyz.shape[1]), -rho * trA),
                            -rho * (A @ u + u * trA) - b[:, None],
                            -((u * gradE).sum(0) + (E + p) * trA + b @ u)[None]])
    NP = N ** 3
    sl = slice(13 * NP, 14 * NP)  # the centre element of the 3 x 3 x 3 box
    for v in range(5):
        np.testing.assert_allclose(R[v, sl], exact[v, sl], rtol=1e-11, atol=1e-11 * np.abs(exact[v]).max(),
                                   err_msg="variable %d" % v)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("w", [0.0, 0.4])
def test_rusanov_dissipation_coefficient_gpu(ch, oracle_mod, torch_dev, precision, w):
    """Closed-form pin of the interface flux of both paths, no oracle values:
    two contact discontinuities in a periodic box (density rho_L for x < 1/2,
    rho_R above, uniform p and velocity (w, 0, 0)); by discrete conservation
    the quadrature sum of the mass residual over the rho_L half is
    lambda (rho_R - rho_L) A with lambda = |w| + max(c_L, c_R) (the oracle's
    pin, same state).  Mixed path: background at rest with the same
    pressure, so the FP32 part carries the whole jump; bound 1e-6 relative."""
    torch = torch_dev
    Ly, Lz, gam, p = 0.8, 0.6, 5.0 / 3.0, 1.2
    N = 4
    m = box_mesh(4, 3, 3, lengths=(1.0, Ly, Lz), periodic=(True,) * 3, curve=0.02)
    cm = ch.mesh_from_arrays(m, N).upload()
    xyz, wJ = cm.solpts()
    rL, rR = 0.7, 1.6
    left = np.repeat(xyz[0].reshape(-1, N ** 3).mean(1) < 0.5, N ** 3)
    rho = np.where(left, rL, rR)
    z = np.zeros_like(rho)
    Q = np.stack([rho, rho * w, z, z, p / (gam - 1) + 0.5 * rho * w * w])
    prec = ch.CHORUS_MIXED if precision == "mixed" else ch.CHORUS_FP64
    phys = ch.physics(gamma=gam, precision=prec)
    ws = cm.workspace(phys)
    if prec == ch.CHORUS_MIXED:
        Q0 = np.stack([np.ones_like(rho), z, z, z, np.full_like(rho, p / (gam - 1))])
        ch.chorus_set_background(cm, phys, torch.from_numpy(np.ascontiguousarray(Q0)).cuda(), ws)
    Qd = torch.from_numpy(np.ascontiguousarray(Q)).cuda()
    Rd = torch.empty_like(Qd)
    ch.chorus_sd_residual(cm, phys, Qd, Rd, ws)
    torch.cuda.synchronize()
    R = Rd.cpu().numpy()
    lam = abs(w) + max(np.sqrt(gam * p / rL), np.sqrt(gam * p / rR))
    expect = lam * (rR - rL) * Ly * Lz
    tol = (1e-12 if precision == "fp64" else 1e-6) * abs(expect)
    assert abs((wJ * R[0])[left].sum() - expect) <= tol, ((wJ * R[0])[left].sum(), expect)
    assert abs((wJ * R[0])[~left].sum() + expect) <= tol


@pytest.mark.parametrize("N", [3, 4])
def test_br1_common_solution_is_the_average_gpu(ch, oracle_mod, torch_dev, N):
    """Closed-form pin of the library's BR1 gradients (the closure features,
    FP32 output), no oracle values: a piecewise-constant density on an affine
    periodic box (0.7 for x < 1/2, 1.6 above); each element's quadrature
    integral of d rho/dx is (rho_R - rho_L) A / 2, signed by the side of the
    jump, for the elements touching the jumps at x = 0 and 1/2 (the common
    value is the average), and the y and z components vanish (the oracle's
    pin, same state)."""
    torch = torch_dev
    Ly, Lz, gam, p = 0.8, 0.6, 5.0 / 3.0, 1.2
    rL, rR, A = 0.7, 1.6, (Ly / 3) * (Lz / 3)
    m = box_mesh(4, 3, 3, lengths=(1.0, Ly, Lz), periodic=(True,) * 3)
    cm = ch.mesh_from_arrays(m, N).upload()
    NP = N ** 3
    xyz, wJ = cm.solpts()
    cx = xyz[0].reshape(-1, NP).mean(1)
    rho = np.repeat(np.where(cx < 0.5, rL, rR), NP)
    z = np.zeros_like(rho)
    Q = np.stack([rho, z, z, z, np.full_like(rho, p / (gam - 1))])
    phys = ch.physics(gamma=gam)
    X = torch.empty((cm.n_solpts, 20), dtype=torch.float32, device="cuda")
    ch.chorus_closure_features(cm, phys, torch.from_numpy(np.ascontiguousarray(Q)).cuda(), X, cm.workspace(phys))
    torch.cuda.synchronize()
    G = X.cpu().numpy().astype(np.float64)[:, 5:8].T  # d rho / dx_c
    integ = (G * wJ[None]).reshape(3, -1, NP).sum(2)
    col = np.floor(cx * 4).astype(int)
    want = np.array([-0.5, 0.5, 0.5, -0.5])[col] * (rR - rL) * A
    np.testing.assert_allclose(integ[0], want, rtol=1e-5, atol=1e-7)
    np.testing.assert_allclose(integ[1:], 0.0, atol=1e-7)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_bottom_flux_enters_through_the_inner_wall_gpu(ch, oracle_mod, torch_dev, precision):
    """Closed-form pin of the inner-wall energy flux on both paths (the
    oracle's pin, same state): for a polytrope at rest with kappa =
    kappa_r = 0 the quadrature sum of the change of the energy residual
    caused by F_bottom is F_bottom times the inner wall's area (4 pi R_i^2
    within the hex20 surface approximation) and mass and momentum do not
    change.  Mixed path: the state is its own background, so the prescribed
    flux sits in the FP64 background residual."""
    torch = torch_dev
    beta = 0.7
    ri, ro = beta / (1 - beta), 1 / (1 - beta)
    m = cubed_sphere_shell(4, 2, ri, ro)
    om = oracle_mod.OracleMesh(m, 3)
    Q, pars = om.polytrope(beta, 1.0)
    cm = ch.mesh_from_arrays(m, 3).upload()
    _, wJ = cm.solpts()
    prec = ch.CHORUS_MIXED if precision == "mixed" else ch.CHORUS_FP64
    f = 0.37
    Qd = torch.from_numpy(np.ascontiguousarray(Q.reshape(5, -1))).cuda()
    out = []
    for fb in (f, 0.0):
        phys = ch.physics(GM=pars["GM"], nu=1e-3, F_bottom=fb, precision=prec)
        ws = cm.workspace(phys)
        if prec == ch.CHORUS_MIXED:
            ch.chorus_set_background(cm, phys, Qd, ws)
        R = torch.empty_like(Qd)
        ch.chorus_sd_residual(cm, phys, Qd, R, ws)
        torch.cuda.synchronize()
        out.append(R.cpu().numpy())
    dE = (wJ * (out[0][4] - out[1][4])).sum()
    assert abs(dE / (f * 4 * np.pi * ri ** 2) - 1.0) < 2e-3, dE / (f * 4 * np.pi * ri ** 2)
    scale = np.abs(out[1][:4]).max()
    assert np.abs(out[0][:4] - out[1][:4]).max() <= 1e-12 * scale


@pytest.mark.parametrize("N", [3, 4])
def test_outer_wall_temperature_enters_the_gradient_gpu(ch, oracle_mod, torch_dev, N):
    """Closed-form pin of the library's outer-wall state (the oracle's pin,
    same state, through the BR1 gradients of the closure features): on an
    affine box walled all round (outer walls) with a uniform state at rest,
    each element's quadrature integral of dE/dx_c is the sum over its wall
    faces of (E_b - E) n_c A, E_b = rho R T_top / (gamma - 1); the density
    and momentum gradients vanish."""
    torch = torch_dev
    gam, rho, p, T_top = 5.0 / 3.0, 1.1, 1.3, 0.9
    lengths = (1.0, 1.2, 0.9)
    m = box_mesh(3, 3, 3, lengths=lengths, bc=2)
    cm = ch.mesh_from_arrays(m, N).upload()
    NP = N ** 3
    xyz, wJ = cm.solpts()
    n = xyz.shape[1]
    Q = np.stack([np.full(n, rho), np.zeros(n), np.zeros(n), np.zeros(n), np.full(n, p / (gam - 1))])
    phys = ch.physics(gamma=gam, T_top=T_top)
    X = torch.empty((n, 20), dtype=torch.float32, device="cuda")
    ch.chorus_closure_features(cm, phys, torch.from_numpy(np.ascontiguousarray(Q)).cuda(), X, cm.workspace(phys))
    torch.cuda.synchronize()
    G = X.cpu().numpy().astype(np.float64)[:, 5:20].T
    integ = (G * wJ[None]).reshape(15, -1, NP).sum(2)
    cent = xyz.reshape(3, -1, NP).mean(2)
    Eb, E = rho * T_top / (gam - 1), p / (gam - 1)
    h = np.asarray(lengths) / 3
    want = np.zeros((3, cent.shape[1]))
    for c in range(3):
        idx = np.floor(cent[c] / h[c]).astype(int)
        want[c] = ((idx == 2).astype(float) - (idx == 0).astype(float)) * (Eb - E) * np.prod(h) / h[c]
    np.testing.assert_allclose(integ[12:15], want, rtol=1e-5, atol=1e-7)
    np.testing.assert_allclose(integ[0:12], 0.0, atol=1e-7)

def gpu_residual_prec(ch, torch, cm, phys, Q, Q0=None):
    """Residual on either path; the mixed path takes the background Q0 (a
    state at rest)."""
    Qd = torch.from_numpy(np.ascontiguousarray(Q.reshape(5, -1))).cuda()
    ws = cm.workspace(phys)
    if phys.precision == ch.CHORUS_MIXED:
        ch.chorus_set_background(cm, phys, torch.from_numpy(np.ascontiguousarray(Q0.reshape(5, -1))).cuda(), ws)
    R = torch.empty_like(Qd)
    ch.chorus_sd_residual(cm, phys, Qd, R, ws)
    torch.cuda.synchronize()
    return R.cpu().numpy()


def uniform_rest(n, rho, p, gam):
    z = np.zeros(n)
    return np.stack([np.full(n, rho), z, z, z, np.full(n, p / (gam - 1))])


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("N", [3, 4])
@pytest.mark.parametrize("bc", [1, 2])
def test_stress_free_wall_traction_gpu(ch, oracle_mod, torch_dev, precision, N, bc):
    """Closed-form pin of the stress-free walls (Section 5) on both paths,
    no oracle values (the oracle's pin, same state): on the affine slab
    walled in x with u = (c x (L - x), a x, b x) at uniform rho and p, each
    element's quadrature integral of the viscous residual R(nu) - R(0) is
    the divergence theorem for tau and u.tau plus, on the wall elements,
    the dropped tangential traction and viscous work.  Mixed path: the
    background is the uniform state at rest, so the FP32 part carries the
    whole velocity field; bound 1e-5 of the largest integral."""
    from chorus_inputs import walled_slab_mesh
    import closed_forms as cf
    m = walled_slab_mesh(cf.SLAB["nx"], cf.SLAB["ny"], cf.SLAB["nz"], cf.SLAB["lengths"], bc, bc)
    cm = ch.mesh_from_arrays(m, N).upload()
    xyz, wJ = cm.solpts()
    t = cf.TRACTION
    prec = ch.CHORUS_MIXED if precision == "mixed" else ch.CHORUS_FP64
    Q = cf.traction_state(xyz)
    Q0 = uniform_rest(xyz.shape[1], t["rho"], t["p"], t["gamma"])
    R1 = gpu_residual_prec(ch, torch_dev, cm, ch.physics(gamma=t["gamma"], nu=t["nu"], precision=prec), Q, Q0)
    R0 = gpu_residual_prec(ch, torch_dev, cm, ch.physics(gamma=t["gamma"], precision=prec), Q, Q0)
    integ = ((R1 - R0) * wJ[None]).reshape(5, -1, N ** 3).sum(2)
    want = cf.traction_expected(xyz, N ** 3)
    rel = 1e-11 if precision == "fp64" else 1e-5
    scale = np.abs(want[1:]).max()
    err = np.abs(integ[1:] - want[1:]).max()
    print("traction %s N=%d bc=%d: max |err| / scale = %.2e (bound %.0e)" % (precision, N, bc, err / scale, rel))
    assert err <= rel * scale
    assert np.abs(integ[0]).max() <= rel * scale
    for wrong in ("full", "none"):
        assert np.abs(cf.traction_expected(xyz, N ** 3, wall=wrong) - want).max() > 100 * rel * scale


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("N", [3, 4])
def test_wall_energy_fluxes_gpu(ch, oracle_mod, torch_dev, precision, N):
    """Closed-form pin of the wall energy fluxes (Section 5) on both paths
    (the oracle's pin, same state): on the affine slab with the inner wall
    at x = 0 and the outer wall at x = L, at rest with rho and p linear in
    x, each element's quadrature integral of the energy residual's
    diffusive part is the conductive flux through its x-faces, F_bottom
    entering through the inner wall and the interior flux leaving through
    the outer wall (T_top = the interior wall temperature).  Mixed path:
    the background is the uniform state (r0, p0) at rest; bound 1e-5."""
    from chorus_inputs import walled_slab_mesh
    import closed_forms as cf
    m = walled_slab_mesh(cf.SLAB["nx"], cf.SLAB["ny"], cf.SLAB["nz"], cf.SLAB["lengths"], 1, 2)
    cm = ch.mesh_from_arrays(m, N).upload()
    xyz, wJ = cm.solpts()
    t = cf.CONDUCTION
    prec = ch.CHORUS_MIXED if precision == "mixed" else ch.CHORUS_FP64
    Q = cf.conduction_state(xyz)
    Q0 = uniform_rest(xyz.shape[1], t["r0"], t["p0"], t["gamma"])
    kw = dict(gamma=t["gamma"], R_gas=t["R_gas"], T_top=cf.conduction_T_top(), precision=prec)
    R1 = gpu_residual_prec(ch, torch_dev, cm, ch.physics(kappa=t["kappa"], kappa_r=t["kappa_r"],
                                                         F_bottom=t["F_bottom"], **kw), Q, Q0)
    R0 = gpu_residual_prec(ch, torch_dev, cm, ch.physics(**kw), Q, Q0)
    integ = ((R1 - R0) * wJ[None]).reshape(5, -1, N ** 3).sum(2)
    want = cf.conduction_expected(xyz, N ** 3)
    rel = 1e-11 if precision == "fp64" else 1e-5
    scale = np.abs(want).max()
    err = np.abs(integ[4] - want).max()
    print("wall energy %s N=%d: max |err| / scale = %.2e (bound %.0e)" % (precision, N, err / scale, rel))
    assert err <= rel * scale
    assert np.abs(integ[:4]).max() <= rel * scale
    for wrong in ("adiabatic", "flipped"):
        assert np.abs(cf.conduction_expected(xyz, N ** 3, outer=wrong) - want).max() > 100 * rel * scale


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_design_order_isentropic_vortex_gpu(ch, oracle_mod, torch_dev, precision):
    """Design order of the library's nonlinear inviscid scheme on both paths
    (the oracle's pin, same runs): the isentropic vortex advected on curved
    periodic slabs, error at t = 1 over the vortex disc at h = L/12 and
    L/24; rate > N - 0.5 for N = 2, 4 and > 2.4 for N = 3.  Mixed path: the
    background is the uniform far-field state at rest, so the vortex and
    the mean flow are the FP32 perturbation."""
    from chorus_inputs import warped_slab_mesh
    import closed_forms as cf
    torch = torch_dev
    v = cf.VORTEX
    prec = ch.CHORUS_MIXED if precision == "mixed" else ch.CHORUS_FP64
    phys = ch.physics(gamma=v["gamma"], precision=prec)

    def run(N, n):
        cm = ch.mesh_from_arrays(warped_slab_mesh(n, v["length"], v["amp"]), N).upload()
        xyz, wJ = cm.solpts()
        ws = cm.workspace(phys)
        if prec == ch.CHORUS_MIXED:
            Q0 = uniform_rest(xyz.shape[1], 1.0, 1.0, v["gamma"])
            ch.chorus_set_background(cm, phys, torch.from_numpy(Q0).cuda(), ws)
        Qd = torch.from_numpy(np.ascontiguousarray(cf.vortex_state(xyz, 0.0))).cuda()
        steps = cf.vortex_steps(N, n)
        ch.chorus_rk_step(cm, phys, Qd, v["t_end"] / steps, steps, ws)
        torch.cuda.synchronize()
        return cf.vortex_errors(Qd.cpu().numpy(), xyz, wJ)

    for N, bound in ((2, 1.5), (3, 2.4), (4, 3.5)):
        e1, e2 = run(N, 12), run(N, 24)
        rates = np.log2(e1[[0, 1, 2, 4]] / e2[[0, 1, 2, 4]])
        print("vortex %s N=%d: errors %s, rates %s" % (precision, N, e2, rates))
        assert (rates > bound).all(), (N, e1, e2, rates)


@pytest.mark.parametrize("N", [2, 3, 4, 5, 6])
@pytest.mark.parametrize("dims", [(1, 1, 1), (1, 1, 3)])
def test_residual_parity_fewer_elements_than_a_block(ch, oracle_mod, torch_dev, N, dims):
    """One element (far-field faces all round) and three elements (periodic
    along z): fewer elements than one block of the flux pass holds at N = 2
    (8) and a ragged last block at N = 3 (2 per block); residual and three
    RK3 steps."""
    m = box_mesh(*dims, lengths=(1.0, 1.0, float(dims[2])), periodic=(False, False, dims[2] > 1))
    om = oracle_mod.OracleMesh(m, N)
    xyz, _ = om.solpts()
    x, y, z = xyz
    Q = np.stack([1 + 0.2 * np.sin(2 * np.pi * (x + y)), 0.3 + 0.1 * np.cos(2 * np.pi * z / dims[2]),
                  -0.2 + 0.05 * np.sin(2 * np.pi * x), 0.1 * np.cos(2 * np.pi * y), 2.5 + 0.1 * np.sin(2 * np.pi * z)])
    phys = ch.physics(GM=1.0, omega=0.5, nu=1e-2, kappa=1e-2, kappa_r=1e-3,
                      bc_state=[1.0, 0.3, -0.2, 0.1, 2.5])
    cm = ch.mesh_from_arrays(m, N).upload()
    R = gpu_residual(ch, torch_dev, cm, phys, Q)
    op = ora_phys(oracle_mod, phys)
    Qo = Q.reshape(5, om.E, om.np)
    Rp = perturbed_oracle(oracle_mod, m, N).residual(op, ulp_perturb(Qo))
    assert_parity(R, om.residual(op, Qo), Rp, "E=%d N=%d" % (om.E, N))
    torch = torch_dev
    Qd = torch.from_numpy(np.ascontiguousarray(Q.reshape(5, -1))).cuda()
    ch.chorus_rk_step(cm, phys, Qd, 1e-3, 3, cm.workspace(phys))
    torch.cuda.synchronize()
    Qr = om.rk3(op, Qo, 1e-3, 3).reshape(5, -1)
    Qp = perturbed_oracle(oracle_mod, m, N).rk3(op, ulp_perturb(Qo), 1e-3, 3).reshape(5, -1)
    Q0 = Q.reshape(5, -1)
    assert_parity(Qd.cpu().numpy() - Q0, Qr - Q0, Qp - Q0, "rk3 E=%d N=%d" % (om.E, N))


@pytest.mark.parametrize("rot", range(24))
def test_residual_parity_orientations(ch, oracle_mod, torch_dev, rot):
    m = two_element_mesh(rot)
    om = oracle_mod.OracleMesh(m, 3)
    xyz, _ = om.solpts()
    x, y, z = xyz
    Q = np.stack([1 + 0.1 * np.sin(x + 2 * y), 0.1 * np.cos(z), 0.05 * x, -0.02 * y * z, 2.5 + 0.1 * np.cos(x * y)])
    phys = ch.physics(nu=1e-2, kappa=1e-2, GM=0.5, omega=0.3, bc_state=(1, 0, 0, 0, 2.5))
    cm = ch.mesh_from_arrays(m, 3).upload()
    R = gpu_residual(ch, torch_dev, cm, phys, Q)
    op = ora_phys(oracle_mod, phys)
    Qo = Q.reshape(5, om.E, om.np)
    Rp = perturbed_oracle(oracle_mod, m, 3).residual(op, ulp_perturb(Qo))
    assert_parity(R, om.residual(op, Qo), Rp, "rot %d" % rot)


def test_rk3_ten_steps_parity_c1(ch, oracle_mod, torch_dev):
    """10 SSP-RK3 steps on the 288-hex N=3 shell (the plain FP64 config)."""
    torch = torch_dev
    m, om, Q, phys = shell_case(oracle_mod, ch, 4, 3, 3, amp=1e-4)
    cm = ch.mesh_from_arrays(m, 3).upload()
    dt = 0.02
    Qd = torch.from_numpy(np.ascontiguousarray(Q.reshape(5, -1))).cuda()
    ws = cm.workspace(phys)
    ch.chorus_rk_step(cm, phys, Qd, dt, 10, ws)
    torch.cuda.synchronize()
    Qg = Qd.cpu().numpy()
    op = ora_phys(oracle_mod, phys)
    Qr = om.rk3(op, Q, dt, 10).reshape(5, -1)
    Qp = perturbed_oracle(oracle_mod, m, 3).rk3(op, ulp_perturb(Q), dt, 10).reshape(5, -1)
    # compare the change over the run (the state itself is background-sized)
    Q0 = Q.reshape(5, -1)
    assert_parity(Qg - Q0, Qr - Q0, Qp - Q0, "rk3 C1")


def test_deterministic_and_conservative(ch, oracle_mod, torch_dev):
    torch = torch_dev
    m, om, Q, phys = shell_case(oracle_mod, ch, 4, 3, 3, amp=1e-3)
    cm = ch.mesh_from_arrays(m, 3).upload()
    ws = cm.workspace(phys)
    outs = []
    for _ in range(2):
        Qd = torch.from_numpy(np.ascontiguousarray(Q.reshape(5, -1))).cuda()
        ch.chorus_rk_step(cm, phys, Qd, 0.02, 5, ws)
        torch.cuda.synchronize()
        outs.append(Qd.cpu().numpy())
    assert np.array_equal(outs[0], outs[1])
    Q0 = torch.from_numpy(np.ascontiguousarray(Q.reshape(5, -1))).cuda()
    s0 = ch.chorus_conserved_sums(cm, Q0, ws)
    s1 = ch.chorus_conserved_sums(cm, torch.from_numpy(outs[0]).cuda(), ws)
    assert abs(s1[0] - s0[0]) < 1e-14 * abs(s0[0])
    # the sums agree with the oracle's serial sums
    np.testing.assert_allclose(s0, om.sums(Q), rtol=1e-13, atol=1e-13)


def test_check_finite_flag(ch, oracle_mod, torch_dev):
    torch = torch_dev
    m, om, Q, phys = shell_case(oracle_mod, ch, 2, 1, 3)
    cm = ch.mesh_from_arrays(m, 3).upload()
    phys.flags = ch.CHORUS_CHECK_FINITE
    Qb = Q.reshape(5, -1).copy()
    Qb[0, 5] = -1.0  # negative density, set from the host
    Qd = torch.from_numpy(Qb).cuda()
    R = torch.empty_like(Qd)
    with pytest.raises(ch.ChorusError) as ei:
        ch.chorus_sd_residual(cm, phys, Qd, R, cm.workspace(phys))
    assert ei.value.status == -5



@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_rk_step_argument_edges(ch, oracle_mod, torch_dev, precision):
    """Zero steps leave the state bitwise unchanged; a negative step count or
    a non-finite dt is an argument error (CHORUS_EINVAL) that leaves the
    state untouched; the mixed path without a background for this workspace
    is a call-order error (CHORUS_ESTATE)."""
    torch = torch_dev
    m, om, Q, phys = shell_case(oracle_mod, ch, 2, 2, 4)
    if precision == "mixed":
        phys.precision = ch.CHORUS_MIXED
    cm = ch.mesh_from_arrays(m, 4).upload()
    ws = cm.workspace(phys)
    Qd = torch.from_numpy(np.ascontiguousarray(Q.reshape(5, -1))).cuda()
    if precision == "mixed":
        with pytest.raises(ch.ChorusError) as ei:
            ch.chorus_rk_step(cm, phys, Qd, 0.01, 1, ws)
        assert ei.value.status == -6
        Q0 = torch.from_numpy(np.ascontiguousarray(om.polytrope(0.7, 1.0)[0].reshape(5, -1))).cuda()
        ch.chorus_set_background(cm, phys, Q0, ws)
        # a background with momentum is rejected and unregisters the previous one
        with pytest.raises(ch.ChorusError) as ei:
            ch.chorus_set_background(cm, phys, Qd.clone(), ws)
        assert ei.value.status == -1
        with pytest.raises(ch.ChorusError) as ei:
            ch.chorus_rk_step(cm, phys, Qd, 0.01, 1, ws)
        assert ei.value.status == -6
        ch.chorus_set_background(cm, phys, Q0, ws)
    ch.chorus_rk_step(cm, phys, Qd, 0.01, 0, ws)
    for n, dt in ((-1, 0.01), (1, float("nan")), (1, float("inf"))):
        with pytest.raises(ch.ChorusError) as ei:
            ch.chorus_rk_step(cm, phys, Qd, dt, n, ws)
        assert ei.value.status == -1, (n, dt)
    torch.cuda.synchronize()
    assert np.array_equal(Qd.cpu().numpy(), Q.reshape(5, -1))
    # and a real step after the rejected calls still runs
    ch.chorus_rk_step(cm, phys, Qd, 0.01, 1, ws)
    torch.cuda.synchronize()
    out = Qd.cpu().numpy()
    assert np.isfinite(out).all() and not np.array_equal(out, Q.reshape(5, -1))

def test_full_size_jupiter_workload(ch, oracle_mod, torch_dev):
    """The benchmark workload at full size (41,472 hexes, N=4, 2.65M DOFs),
    built the way bench.py builds it (library shell generator), against the
    oracle on the same mesh from the input generator: residual and one
    SSP-RK3 step at the benchmark's time step."""
    from chorus_inputs import CONFIGS, shell_params_from_config
    torch = torch_dev
    cfg = CONFIGS["jupiter_41k_N4"]
    ri, ro = shell_params_from_config(cfg)
    m = cubed_sphere_shell(cfg["panel_n"], cfg["radial_n"], ri, ro)
    om = oracle_mod.OracleMesh(m, 4)
    Q, pars = om.polytrope(cfg["beta"], cfg["n_rho"], noise=uniform_noise(om.n_solpts, cfg["seed"]), amp=1e-4)
    cm = ch.chorus_mesh_create(cfg["panel_n"], cfg["radial_n"], 4, ri, ro).upload()
    phys = ch.physics(GM=pars["GM"], omega=cfg["omega"], nu=cfg["nu"], kappa=cfg["kappa"], T_top=pars["chi_o"])
    op = ora_phys(oracle_mod, phys)
    R = gpu_residual(ch, torch, cm, phys, Q)
    Rp = perturbed_oracle(oracle_mod, m, 4).residual(op, ulp_perturb(Q))
    assert_parity(R, om.residual(op, Q), Rp, "jupiter residual")
    dt = cm.stable_dt(phys, Q.reshape(5, -1), cfg["cfl"])
    Qd = torch.from_numpy(np.ascontiguousarray(Q.reshape(5, -1))).cuda()
    ch.chorus_rk_step(cm, phys, Qd, dt, 1, cm.workspace(phys))
    torch.cuda.synchronize()
    Q0 = Q.reshape(5, -1)
    Qr = om.rk3(op, Q, dt, 1).reshape(5, -1)
    Qp = perturbed_oracle(oracle_mod, m, 4).rk3(op, ulp_perturb(Q), dt, 1).reshape(5, -1)
    assert_parity(Qd.cpu().numpy() - Q0, Qr - Q0, Qp - Q0, "jupiter rk3")
